/*
 * VBARMS CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential FP64 implementation of the VBARMS hot path, written from
 * the paper ("Using the VBARMS method in parallel computing", Carpentieri, Liao,
 * Sosonkina, Bonfiglioli, arXiv:1508.02219) to check the GPU library against.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code with the GPU path.
 *
 * Every loop follows the order of the algorithm it restates; there is no blocking,
 * fusion or reordering.  Build with -O2 -ffp-contract=off so that no multiply-add is
 * fused.
 *
 * Readings of passages the paper leaves open (each is also listed in the design notes):
 *  R1 (Sec. 2.1) row j joins the group of row i when cos(r_i, r_j) >= tau, evaluated
 *     exactly as c*c >= tau^2 * |r_i||r_j| with c = |r_i & r_j|; rows are compared with
 *     the seed only; seeds and candidates are visited in ascending order; empty rows
 *     stay singletons.
 *  R2 (Sec. 3, Step 2) S1 = 1/max|a_ij| per row, then S2 = 1/max_i|s1_i a_ij| per column
 *     of the row-scaled matrix; an all-zero row or column gets 1.
 *  R3 (Sec. 2 and Sec. 3, Step 3) natural-order greedy independent set on the quotient
 *     graph of A + A^T, one supernode per group.
 *  R4 (Sec. 3, block ILUT paragraph) a block B (m x n) is dropped iff
 *     ||B||_F / (m n) < t, evaluated as sumsq(B) < (t*m*n)^2 with sumsq summed in
 *     row-major order; applied to L^{-1}F, E U^{-1}, off-diagonal Schur blocks (unless
 *     drop_schur == 0) and the last-level L and off-diagonal U blocks; diagonal blocks
 *     are never dropped.
 *  R5 (Alg. 3) the last level is a block IKJ ILUT in the inherited order; every
 *     structurally present block left of the diagonal is eliminated in ascending
 *     column order, its multiplier is dropped before use if it passes R4.
 *  R6 (Eq. blockperm) every block row carries its diagonal block, zero padded if no
 *     entry of A falls there.
 *  R7 (Sec. 3, Step 3, "weighted greedy") the weighted mode visits supernodes by
 *     descending w_I = ||A_II||_F / sum_J ||A_IJ||_F of the scaled matrix, so rows whose
 *     diagonal block dominates enter the independent set first; ties in ascending I.
 *     The set is still listed in ascending supernode order in P_I.
 *  R8 (Sec. 2 and Sec. 3, Step 3, groups of nodes) with a group limit gmax > 0 an
 *     unmarked supernode v opens a group and its unmarked quotient-graph neighbours join
 *     it in ascending order, each one that keeps the group within gmax rows (larger ones
 *     are skipped, later ones may still join); then the members and all their neighbours
 *     are marked.  gmax = 0 is R3 (v alone).  Groups are listed by their smallest
 *     supernode, members ascending; the group is one dense pivot block D_i (zero padded
 *     where no block is stored), factored exactly by GEPP, and the blocks of L^{-1}F and
 *     E U^{-1} are the group's rows (columns) against one remaining supernode, so R4
 *     tests them at that size.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_OOM (-3)
#define ORC_ERR_SINGULAR (-4)
#define ORC_ERR_STATE (-6)

/* ------------------------------------------------------------------------- */
/* Block sparse row matrix: blocks stored row-major, block columns ascending. */
/* ------------------------------------------------------------------------- */
typedef struct {
    int p, q;       /* block rows / block columns */
    int *rb, *cb;   /* scalar offsets of row blocks [p+1] and column blocks [q+1] */
    int64_t *rp;    /* block row pointer [p+1] */
    int *ci;        /* block column index [nb] */
    int64_t *vo;    /* value offset of every block [nb+1] */
    double *v;      /* values */
    int64_t nb, nb_cap, v_cap;
    int cur_row;
} bmat;

static void *xmalloc(size_t n) {
    void *p = malloc(n ? n : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}
static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s ? s : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}
static void *xrealloc(void *q, size_t n) {
    void *p = realloc(q, n ? n : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

static void bm_init(bmat *a, int p, const int *rb, int q, const int *cb) {
    memset(a, 0, sizeof(*a));
    a->p = p; a->q = q;
    a->rb = xmalloc(sizeof(int) * (p + 1));
    a->cb = xmalloc(sizeof(int) * (q + 1));
    memcpy(a->rb, rb, sizeof(int) * (p + 1));
    memcpy(a->cb, cb, sizeof(int) * (q + 1));
    a->rp = xcalloc(p + 1, sizeof(int64_t));
    a->nb_cap = 16; a->v_cap = 256;
    a->ci = xmalloc(sizeof(int) * a->nb_cap);
    a->vo = xmalloc(sizeof(int64_t) * (a->nb_cap + 1));
    a->v = xmalloc(sizeof(double) * a->v_cap);
    a->vo[0] = 0;
    a->cur_row = 0;
}
static void bm_free(bmat *a) {
    free(a->rb); free(a->cb); free(a->rp); free(a->ci); free(a->vo); free(a->v);
    memset(a, 0, sizeof(*a));
}
static inline int bm_rs(const bmat *a, int i) { return a->rb[i + 1] - a->rb[i]; }
static inline int bm_cs(const bmat *a, int j) { return a->cb[j + 1] - a->cb[j]; }
static inline double *bm_blk(const bmat *a, int64_t k) { return a->v + a->vo[k]; }

/* append block (row = a->cur_row, column j) */
static void bm_push(bmat *a, int j, const double *blk) {
    int m = bm_rs(a, a->cur_row), n = bm_cs(a, j);
    if (a->nb + 1 >= a->nb_cap) {
        a->nb_cap *= 2;
        a->ci = xrealloc(a->ci, sizeof(int) * a->nb_cap);
        a->vo = xrealloc(a->vo, sizeof(int64_t) * (a->nb_cap + 1));
    }
    int64_t need = a->vo[a->nb] + (int64_t)m * n;
    if (need > a->v_cap) {
        while (a->v_cap < need) a->v_cap *= 2;
        a->v = xrealloc(a->v, sizeof(double) * a->v_cap);
    }
    a->ci[a->nb] = j;
    memcpy(a->v + a->vo[a->nb], blk, sizeof(double) * m * n);
    a->vo[a->nb + 1] = need;
    a->nb++;
}
static void bm_end_row(bmat *a) {
    a->cur_row++;
    a->rp[a->cur_row] = a->nb;
}
/* index of block (i, j) or -1 */
static int64_t bm_find(const bmat *a, int i, int j) {
    for (int64_t k = a->rp[i]; k < a->rp[i + 1]; ++k)
        if (a->ci[k] == j) return k;
    return -1;
}

/* sort helper for small int lists */
static int cmp_int(const void *x, const void *y) {
    int a = *(const int *)x, b = *(const int *)y;
    return (a > b) - (a < b);
}

/* ------------------------------------------------------------------------- */
/* Dense kernels on one block                                                */
/* ------------------------------------------------------------------------- */

/* Gaussian elimination with partial pivoting of an m x m row-major block, in place
 * (Sec. 3: block pivots are inverted exactly by GEPP).  The pivot of column k is the
 * first row of largest magnitude; piv[k] is the row swapped with row k.  On exit the
 * strict lower part holds L (unit diagonal) and the upper part U, with P D = L U. */
static int gepp(int m, double *a, int *piv) {
    for (int k = 0; k < m; ++k) {
        int pr = k;
        double amax = fabs(a[k * m + k]);
        for (int r = k + 1; r < m; ++r)
            if (fabs(a[r * m + k]) > amax) { amax = fabs(a[r * m + k]); pr = r; }
        piv[k] = pr;
        if (amax == 0.0) return ORC_ERR_SINGULAR;
        if (pr != k)
            for (int c = 0; c < m; ++c) { double t = a[k * m + c]; a[k * m + c] = a[pr * m + c]; a[pr * m + c] = t; }
        for (int r = k + 1; r < m; ++r) {
            a[r * m + k] = a[r * m + k] / a[k * m + k];
            for (int c = k + 1; c < m; ++c) a[r * m + c] = a[r * m + c] - a[r * m + k] * a[k * m + c];
        }
    }
    return ORC_OK;
}

/* x <- L^{-1} P x for a column vector (all row swaps first, then unit forward substitution) */
static void lu_fwd(int m, const double *lu, const int *piv, double *x) {
    for (int k = 0; k < m; ++k)
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    for (int r = 0; r < m; ++r) {
        double s = x[r];
        for (int q = 0; q < r; ++q) s = s - lu[r * m + q] * x[q];
        x[r] = s;
    }
}
/* x <- U^{-1} x */
static void lu_bwd(int m, const double *lu, double *x) {
    for (int r = m - 1; r >= 0; --r) {
        double s = x[r];
        for (int q = r + 1; q < m; ++q) s = s - lu[r * m + q] * x[q];
        x[r] = s / lu[r * m + r];
    }
}
/* row vector e <- e U^{-1}  (solve x U = e) */
static void row_solve_u(int m, const double *lu, double *e) {
    for (int c = 0; c < m; ++c) {
        double s = e[c];
        for (int q = 0; q < c; ++q) s = s - e[q] * lu[q * m + c];
        e[c] = s / lu[c * m + c];
    }
}
/* row vector e <- e L^{-1} P  (solve z L = e, then undo the row swaps on the columns) */
static void row_solve_lp(int m, const double *lu, const int *piv, double *e) {
    for (int c = m - 1; c >= 0; --c) {
        double s = e[c];
        for (int q = c + 1; q < m; ++q) s = s - e[q] * lu[q * m + c];
        e[c] = s;
    }
    for (int k = m - 1; k >= 0; --k)
        if (piv[k] != k) { double t = e[k]; e[k] = e[piv[k]]; e[piv[k]] = t; }
}

/* drop rule (Sec. 3): ||B||_F / (m n) < t */
static int drop_block(int m, int n, const double *b, double t) {
    double s = 0.0;
    for (int i = 0; i < m * n; ++i) s = s + b[i] * b[i];
    double thr = t * (double)(m * n);
    return s < thr * thr;
}

/* ------------------------------------------------------------------------- */
/* Step 1: angle-based compression (Sec. 2.1) and the VBCSR matrix             */
/* ------------------------------------------------------------------------- */

/* Groups rows whose patterns are close: for each unassigned row i in ascending order,
 * open a group seeded by i and add every later unassigned row j with cos >= tau.
 * Rows sharing no column with i have cosine 0 < tau, so only rows reached through a
 * common column are examined.  Outputs perm (new position -> old row) and bptr. */
int orc_compress(int n, const int64_t *rowptr, const int32_t *col, double tau,
                 int32_t *perm, int32_t *bptr, int32_t *p_out) {
    if (n < 0 || !(tau > 0.0) || !(tau <= 1.0)) return ORC_ERR_ARG;
    int64_t nnz = rowptr[n];
    /* transpose of the pattern: rows of every column */
    int64_t *cp = xcalloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t k = 0; k < nnz; ++k) {
        if (col[k] < 0 || col[k] >= n) { free(cp); return ORC_ERR_ARG; }
        cp[col[k] + 1]++;
    }
    for (int j = 0; j < n; ++j) cp[j + 1] += cp[j];
    int32_t *cr = xmalloc(sizeof(int32_t) * (size_t)(nnz ? nnz : 1));
    int64_t *fill = xmalloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, cp, sizeof(int64_t) * ((size_t)n + 1));
    for (int i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) cr[fill[col[k]]++] = i;
    free(fill);

    const double tau2 = tau * tau;
    int32_t *group = xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t *cnt = xcalloc((size_t)n + 1, sizeof(int64_t));
    int32_t *touched = xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int i = 0; i < n; ++i) group[i] = -1;
    for (int i = 0; i < n; ++i) {
        if (group[i] != -1) continue;
        group[i] = i; /* i seeds a new group */
        int64_t li = rowptr[i + 1] - rowptr[i];
        if (li == 0) continue;
        int nt = 0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int c = col[k];
            for (int64_t t = cp[c]; t < cp[c + 1]; ++t) {
                int j = cr[t];
                if (j <= i) continue;
                if (cnt[j] == 0) touched[nt++] = j;
                cnt[j]++;
            }
        }
        for (int t = 0; t < nt; ++t) {
            int j = touched[t];
            int64_t c = cnt[j];
            cnt[j] = 0;
            if (group[j] != -1) continue;
            int64_t lj = rowptr[j + 1] - rowptr[j];
            if (lj == 0) continue;
            double lhs = (double)c * (double)c;
            double rhs = tau2 * (double)(li * lj);
            if (lhs >= rhs) group[j] = i;
        }
    }
    /* groups in seed order, members ascending */
    int32_t *gsize = xcalloc((size_t)n + 1, sizeof(int32_t));
    for (int i = 0; i < n; ++i) gsize[group[i]]++;
    int32_t *gstart = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int p = 0, pos = 0;
    bptr[0] = 0;
    for (int s = 0; s < n; ++s) {
        if (group[s] != s) { gstart[s] = -1; continue; }
        gstart[s] = pos;
        pos += gsize[s];
        bptr[++p] = pos;
    }
    for (int i = 0; i < n; ++i) perm[gstart[group[i]]++] = i;
    *p_out = p;
    free(cp); free(cr); free(group); free(cnt); free(touched); free(gsize); free(gstart);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Graph-based compression (Sec. 2.2, Alg. 1; readings G1-G4)                */
/* ------------------------------------------------------------------------- */
/* G1 supernodes start as the classes of rows with identical patterns (the checksum step);
 * G2 a supernode X (visited in ascending order of its smallest row) tries, in ascending
 *    order of their smallest rows, the supernodes adjacent to it in the quotient graph of
 *    A + A^T when its visit starts; a supernode already merged away is skipped, and so is a
 *    merge that would give more than 32 rows (the largest block of the GPU library);
 * G3 the merge is kept iff the average block density of the whole ordering after it, nnz(A)
 *    over the elements of all blocks that hold an entry or lie on the diagonal, is still
 *    at least mu, tested as nnz >= mu * elements in FP64;
 * G4 blocks are ordered by their smallest row, rows ascending within a block. */
#define ORC_GRAPH_MAX_BLOCK 32

/* lexicographic comparison of two row patterns (both sorted ascending) */
static const int64_t *g_rp;
static const int32_t *g_ci;
static int cmp_rows(const void *x, const void *y) {
    int a = *(const int *)x, b = *(const int *)y;
    int64_t la = g_rp[a + 1] - g_rp[a], lb = g_rp[b + 1] - g_rp[b];
    int64_t l = la < lb ? la : lb;
    for (int64_t k = 0; k < l; ++k) {
        int ca = g_ci[g_rp[a] + k], cb = g_ci[g_rp[b] + k];
        if (ca != cb) return (ca > cb) - (ca < cb);
    }
    if (la != lb) return (la > lb) - (la < lb);
    return (a > b) - (a < b);
}

/* elements of all blocks that hold an entry or lie on the diagonal, for supernode labels
 * g (any labels; sz[label] = rows) -- straight from the definition */
static int64_t graph_block_elements(int n, const int64_t *rowptr, const int32_t *col, const int32_t *g,
                                    const int32_t *sz, int32_t *stamp, int32_t *rows_of, int64_t *rstart) {
    /* rows of every label */
    for (int l = 0; l <= n; ++l) rstart[l] = 0;
    for (int i = 0; i < n; ++i) rstart[g[i] + 1]++;
    for (int l = 0; l < n; ++l) rstart[l + 1] += rstart[l];
    int64_t *fill = xmalloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(fill, rstart, sizeof(int64_t) * ((size_t)n + 1));
    for (int i = 0; i < n; ++i) rows_of[fill[g[i]]++] = i;
    free(fill);
    for (int l = 0; l < n; ++l) stamp[l] = -1;
    int64_t elems = 0;
    for (int I = 0; I < n; ++I) {
        if (rstart[I] == rstart[I + 1]) continue;
        /* the diagonal block always counts */
        stamp[I] = I;
        elems += (int64_t)sz[I] * sz[I];
        for (int64_t t = rstart[I]; t < rstart[I + 1]; ++t) {
            int i = rows_of[t];
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                int J = g[col[k]];
                if (stamp[J] != I) {
                    stamp[J] = I;
                    elems += (int64_t)sz[I] * sz[J];
                }
            }
        }
    }
    return elems;
}

int orc_graph_compress(int n, const int64_t *rowptr, const int32_t *col, double mu,
                       int32_t *perm, int32_t *bptr, int32_t *p_out) {
    if (n < 0 || !(mu > 0.0) || !(mu <= 1.0)) return ORC_ERR_ARG;
    int64_t nnz = rowptr[n];
    for (int64_t k = 0; k < nnz; ++k)
        if (col[k] < 0 || col[k] >= n) return ORC_ERR_ARG;
    /* G1: identical patterns (sort rows by pattern, equal neighbours join) */
    int32_t *order = xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int i = 0; i < n; ++i) order[i] = i;
    g_rp = rowptr; g_ci = col;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_rows);
    int32_t *g = xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int t = 0; t < n; ++t) {
        int i = order[t];
        g[i] = i;
        if (t > 0) {
            int j = order[t - 1];
            int64_t li = rowptr[i + 1] - rowptr[i], lj = rowptr[j + 1] - rowptr[j];
            if (li > 0 && li == lj && memcmp(col + rowptr[i], col + rowptr[j], sizeof(int32_t) * li) == 0)
                g[i] = g[j] < i ? g[j] : i;
        }
    }
    /* labels = smallest row of the class (the sort put equal patterns next to each other
     * in ascending row order, so g[j] of the first of a run is its smallest row) */
    int32_t *sz = xcalloc((size_t)n + 1, sizeof(int32_t));
    for (int i = 0; i < n; ++i) sz[g[i]]++;
    /* A + A^T adjacency of rows */
    int64_t *ap = xcalloc((size_t)n + 1, sizeof(int64_t));
    for (int i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) { ap[i + 1]++; ap[col[k] + 1]++; }
    for (int i = 0; i < n; ++i) ap[i + 1] += ap[i];
    int32_t *adj = xmalloc(sizeof(int32_t) * (size_t)(2 * nnz + 1));
    int64_t *af = xmalloc(sizeof(int64_t) * ((size_t)n + 1));
    memcpy(af, ap, sizeof(int64_t) * ((size_t)n + 1));
    for (int i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) { adj[af[i]++] = col[k]; adj[af[col[k]]++] = i; }
    free(af);
    int32_t *stamp = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *rows_of = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int64_t *rstart = xmalloc(sizeof(int64_t) * ((size_t)n + 2));
    int32_t *cand = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *mark = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *gtry = xmalloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *first = xmalloc(sizeof(int32_t) * ((size_t)n + 1)); /* smallest row of every label */
    for (int l = 0; l < n; ++l) { mark[l] = -1; first[l] = l; }
    /* G2/G3: visit supernodes in ascending order of their smallest row */
    for (int X = 0; X < n; ++X) {
        if (g[X] != X || sz[X] == 0) continue; /* not a label, or merged away */
        int nc = 0;
        for (int i = 0; i < n; ++i) {
            if (g[i] != X) continue;
            for (int64_t k = ap[i]; k < ap[i + 1]; ++k) {
                int Z = g[adj[k]];
                if (Z != X && mark[Z] != X) { mark[Z] = X; cand[nc++] = Z; }
            }
        }
        /* ascending smallest row (labels keep their smallest row in first[]) */
        for (int a = 1; a < nc; ++a) {
            int v = cand[a], b = a - 1;
            while (b >= 0 && first[cand[b]] > first[v]) { cand[b + 1] = cand[b]; --b; }
            cand[b + 1] = v;
        }
        for (int c = 0; c < nc; ++c) {
            int Z = cand[c];
            if (sz[Z] == 0) continue;                              /* merged away meanwhile */
            if (sz[X] + sz[Z] > ORC_GRAPH_MAX_BLOCK) continue;
            for (int i = 0; i < n; ++i) gtry[i] = g[i] == Z ? X : g[i];
            int32_t sx = sz[X], szz = sz[Z];
            sz[X] = sx + szz; sz[Z] = 0;
            int64_t el = graph_block_elements(n, rowptr, col, gtry, sz, stamp, rows_of, rstart);
            if ((double)nnz >= mu * (double)el) {
                memcpy(g, gtry, sizeof(int32_t) * (size_t)n);
                if (first[Z] < first[X]) first[X] = first[Z];
            } else {
                sz[X] = sx; sz[Z] = szz;
            }
        }
    }
    /* G4: blocks by smallest row, rows ascending */
    int p = 0;
    for (int l = 0; l < n; ++l) mark[l] = -1;
    for (int i = 0; i < n; ++i) if (mark[g[i]] < 0) mark[g[i]] = p++;   /* rank by smallest row */
    int64_t *bs = xcalloc((size_t)p + 1, sizeof(int64_t));
    for (int i = 0; i < n; ++i) bs[mark[g[i]] + 1]++;
    for (int b = 0; b < p; ++b) bs[b + 1] += bs[b];
    for (int b = 0; b <= p; ++b) bptr[b] = (int32_t)bs[b];
    for (int i = 0; i < n; ++i) perm[bs[mark[g[i]]]++] = i;
    *p_out = p;
    free(order); free(g); free(sz); free(ap); free(adj); free(stamp); free(rows_of); free(rstart);
    free(cand); free(mark); free(gtry); free(first); free(bs);
    return ORC_OK;
}

/* Permuted block matrix P_B A P_B^T (Eq. blockperm): block (I,J) exists iff an entry of
 * A falls in it; the diagonal block always exists (R6); missing entries are zero. */
static void build_vbcsr(int n, const int64_t *rowptr, const int32_t *col, const double *val,
                        const int32_t *perm, const int32_t *bptr, int p, bmat *out) {
    int32_t *inv = xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int32_t *blk = xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int k = 0; k < n; ++k) inv[perm[k]] = k;
    for (int b = 0; b < p; ++b)
        for (int k = bptr[b]; k < bptr[b + 1]; ++k) blk[k] = b;
    bm_init(out, p, bptr, p, bptr);
    int *mark = xmalloc(sizeof(int) * (size_t)(p ? p : 1));
    for (int b = 0; b < p; ++b) mark[b] = -1;
    int *list = xmalloc(sizeof(int) * (size_t)(p ? p : 1));
    double *row = NULL;
    int64_t row_cap = 0;
    for (int I = 0; I < p; ++I) {
        int m = bptr[I + 1] - bptr[I];
        int nl = 0;
        list[nl++] = I;
        mark[I] = I;
        for (int r = bptr[I]; r < bptr[I + 1]; ++r) {
            int orow = perm[r];
            for (int64_t k = rowptr[orow]; k < rowptr[orow + 1]; ++k) {
                int J = blk[inv[col[k]]];
                if (mark[J] != I) { mark[J] = I; list[nl++] = J; }
            }
        }
        qsort(list, nl, sizeof(int), cmp_int);
        /* offsets of every listed block inside a temporary row buffer */
        int64_t width = 0;
        for (int t = 0; t < nl; ++t) width += bptr[list[t] + 1] - bptr[list[t]];
        if (width * m > row_cap) { row_cap = width * m; row = xrealloc(row, sizeof(double) * row_cap); }
        memset(row, 0, sizeof(double) * width * m);
        /* block offset lookup through mark[] reuse: store position in a second pass */
        int64_t *boff = xmalloc(sizeof(int64_t) * (size_t)nl);
        int64_t acc = 0;
        for (int t = 0; t < nl; ++t) { boff[t] = acc; acc += (int64_t)m * (bptr[list[t] + 1] - bptr[list[t]]); }
        for (int r = bptr[I]; r < bptr[I + 1]; ++r) {
            int orow = perm[r];
            for (int64_t k = rowptr[orow]; k < rowptr[orow + 1]; ++k) {
                int c = inv[col[k]];
                int J = blk[c];
                int lo = 0, hi = nl - 1;
                while (lo < hi) { int mid = (lo + hi) / 2; if (list[mid] < J) lo = mid + 1; else hi = mid; }
                int nJ = bptr[J + 1] - bptr[J];
                row[boff[lo] + (int64_t)(r - bptr[I]) * nJ + (c - bptr[J])] = val[k];
            }
        }
        for (int t = 0; t < nl; ++t) bm_push(out, list[t], row + boff[t]);
        bm_end_row(out);
        free(boff);
    }
    free(row); free(mark); free(list); free(inv); free(blk);
}

/* ------------------------------------------------------------------------- */
/* One level of the partial block factorization (Sec. 3, Steps 2-4)          */
/* ------------------------------------------------------------------------- */
typedef struct {
    int p, n;            /* supernodes / scalar size of A_l */
    int nis, n_is;       /* groups (pivot blocks of D) / IS scalar size */
    int nis_sn;          /* supernodes in the groups */
    bmat A;              /* A_l as received (unscaled) */
    bmat As;             /* S1 A_l S2 */
    double *s1, *s2;     /* scaling */
    int *is_list;        /* IS supernodes: the members of group 0, group 1, ... (R8) */
    int *gptr;           /* [nis+1] group g holds is_list[gptr[g] .. gptr[g+1]) */
    int *rest_list;      /* remaining supernodes ascending */
    double *dlu;         /* LU of the IS diagonal blocks, concatenated in IS order */
    int64_t *dlu_off;    /* [nis+1] */
    int *dpiv;           /* pivots, concatenated (offsets = scalar offsets of IS blocks) */
    int *is_rb;          /* scalar offsets of the groups [nis+1] */
    int *rest_rb;        /* scalar offsets of remaining blocks [nrest+1] */
    int *is_rows;        /* [n_is] level row of every row of D, group by group */
    int *rest_rows;      /* [n - n_is] level row of every row of C */
    bmat G;              /* L^{-1} P F  (IS rows, remaining columns) */
    bmat W;              /* E U^{-1}    (remaining rows, IS columns) */
} olevel;

typedef struct {
    int n;               /* original size */
    int p;               /* supernodes after compression */
    int32_t *perm, *bptr;
    int nlev;            /* levels actually factored (<= requested) */
    olevel *lev;
    bmat last;           /* matrix handed to the last-level ILUT */
    bmat L, U;           /* last-level factors: L unit block lower (multipliers), U off-diagonal */
    double *dl;          /* LU of last-level pivot blocks */
    int64_t *dl_off;
    int *dl_piv;
    int status;
    int err_level, err_block;
} orc_t;

/* Step 2 (R2): scaling, applied as (s1_i a_ij) s2_j */
static void level_scale(olevel *L) {
    const bmat *A = &L->A;
    int n = A->rb[A->p];
    L->s1 = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    L->s2 = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    double *cmax = xcalloc((size_t)n + 1, sizeof(double));
    for (int I = 0; I < A->p; ++I) {
        int m = bm_rs(A, I);
        for (int r = 0; r < m; ++r) {
            double mx = 0.0;
            for (int64_t k = A->rp[I]; k < A->rp[I + 1]; ++k) {
                int nJ = bm_cs(A, A->ci[k]);
                const double *b = bm_blk(A, k);
                for (int c = 0; c < nJ; ++c) if (fabs(b[r * nJ + c]) > mx) mx = fabs(b[r * nJ + c]);
            }
            L->s1[A->rb[I] + r] = mx > 0.0 ? 1.0 / mx : 1.0;
        }
    }
    for (int I = 0; I < A->p; ++I) {
        int m = bm_rs(A, I);
        for (int64_t k = A->rp[I]; k < A->rp[I + 1]; ++k) {
            int J = A->ci[k], nJ = bm_cs(A, J);
            const double *b = bm_blk(A, k);
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < nJ; ++c) {
                    double v = fabs(L->s1[A->rb[I] + r] * b[r * nJ + c]);
                    if (v > cmax[A->cb[J] + c]) cmax[A->cb[J] + c] = v;
                }
        }
    }
    for (int j = 0; j < n; ++j) L->s2[j] = cmax[j] > 0.0 ? 1.0 / cmax[j] : 1.0;
    free(cmax);
    bm_init(&L->As, A->p, A->rb, A->q, A->cb);
    double *tmp = NULL;
    int64_t tcap = 0;
    for (int I = 0; I < A->p; ++I) {
        int m = bm_rs(A, I);
        for (int64_t k = A->rp[I]; k < A->rp[I + 1]; ++k) {
            int J = A->ci[k], nJ = bm_cs(A, J);
            if ((int64_t)m * nJ > tcap) { tcap = (int64_t)m * nJ; tmp = xrealloc(tmp, sizeof(double) * tcap); }
            const double *b = bm_blk(A, k);
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < nJ; ++c)
                    tmp[r * nJ + c] = (L->s1[A->rb[I] + r] * b[r * nJ + c]) * L->s2[A->cb[J] + c];
            bm_push(&L->As, J, tmp);
        }
        bm_end_row(&L->As);
    }
    free(tmp);
}

/* Visiting order of the weighted greedy independent set (Sec. 3, Step 3): supernodes by
 * descending weight w_I = ||A_II||_F / sum_J ||A_IJ||_F over the blocks of row I (R7), equal
 * weights in ascending I.  A row without a stored diagonal block has weight 0. */
typedef struct { double w; int I; } wnode;
static int cmp_wnode(const void *x, const void *y) {
    const wnode *a = (const wnode *)x, *b = (const wnode *)y;
    if (a->w > b->w) return -1;
    if (a->w < b->w) return 1;
    return (a->I > b->I) - (a->I < b->I);
}
static void weighted_order(const bmat *A, int *order) {
    int p = A->p;
    wnode *nodes = xmalloc(sizeof(wnode) * (size_t)(p ? p : 1));
    for (int I = 0; I < p; ++I) {
        int m = bm_rs(A, I);
        double diag = 0.0, tot = 0.0;
        for (int64_t k = A->rp[I]; k < A->rp[I + 1]; ++k) {
            int J = A->ci[k], nJ = bm_cs(A, J);
            const double *b = bm_blk(A, k);
            double ss = 0.0;
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < nJ; ++c) ss += b[r * nJ + c] * b[r * nJ + c];
            double f = sqrt(ss);
            tot += f;
            if (J == I) diag = f;
        }
        nodes[I].w = tot > 0.0 ? diag / tot : 0.0;
        nodes[I].I = I;
    }
    qsort(nodes, (size_t)p, sizeof(wnode), cmp_wnode);
    for (int q = 0; q < p; ++q) order[q] = nodes[q].I;
    free(nodes);
}

/* Step 3 (R3, R8): greedy block independent set on the quotient graph of A + A^T,
 * visiting the supernodes in natural order (is_order 0) or by the weights above
 * (is_order 1).  gid[I] receives the group of I in opening order, or -1 for the
 * remaining supernodes; returns the number of groups. */
static int level_groups(const bmat *A, int gmax, int is_order, int *gid) {
    int p = A->p;
    /* transpose pattern so that both (I,J) and (J,I) mark neighbours */
    int64_t *tp = xcalloc((size_t)p + 1, sizeof(int64_t));
    for (int64_t k = 0; k < A->nb; ++k) tp[A->ci[k] + 1]++;
    for (int j = 0; j < p; ++j) tp[j + 1] += tp[j];
    int *tr = xmalloc(sizeof(int) * (size_t)(A->nb ? A->nb : 1));
    int64_t *f = xmalloc(sizeof(int64_t) * ((size_t)p + 1));
    memcpy(f, tp, sizeof(int64_t) * ((size_t)p + 1));
    for (int I = 0; I < p; ++I)
        for (int64_t k = A->rp[I]; k < A->rp[I + 1]; ++k) tr[f[A->ci[k]]++] = I;
    free(f);
    char *marked = xcalloc((size_t)p + 1, 1);
    int *order = xmalloc(sizeof(int) * (size_t)(p ? p : 1));
    int *nbr = xmalloc(sizeof(int) * (2 * (size_t)A->nb + 1));
    int *mem = xmalloc(sizeof(int) * (size_t)(p ? p : 1));
    if (is_order == 1) weighted_order(A, order);
    else for (int I = 0; I < p; ++I) order[I] = I;
    for (int I = 0; I < p; ++I) gid[I] = -1;
    int ng = 0;
    for (int q = 0; q < p; ++q) {
        int v = order[q];
        if (marked[v]) continue;
        int g = ng++, nm = 0, rows = bm_rs(A, v);
        gid[v] = g;
        marked[v] = 1;
        mem[nm++] = v;
        if (gmax > 0) {
            /* neighbours of v, ascending: its row pattern and its column pattern */
            int nn = 0;
            for (int64_t k = A->rp[v]; k < A->rp[v + 1]; ++k) nbr[nn++] = A->ci[k];
            for (int64_t k = tp[v]; k < tp[v + 1]; ++k) nbr[nn++] = tr[k];
            qsort(nbr, (size_t)nn, sizeof(int), cmp_int);
            for (int a = 0; a < nn; ++a) {
                int u = nbr[a];
                if (marked[u]) continue;
                if (rows + bm_rs(A, u) > gmax) continue;
                gid[u] = g;
                marked[u] = 1;
                mem[nm++] = u;
                rows += bm_rs(A, u);
            }
        }
        for (int a = 0; a < nm; ++a) {
            int I = mem[a];
            for (int64_t k = A->rp[I]; k < A->rp[I + 1]; ++k) marked[A->ci[k]] = 1;
            for (int64_t k = tp[I]; k < tp[I + 1]; ++k) marked[tr[k]] = 1;
        }
    }
    free(tp); free(tr); free(marked); free(order); free(nbr); free(mem);
    return ng;
}

/* Steps 3-4 on one level; produces A_{l+1} in *next */
static int level_factor(olevel *L, double t, int drop_schur, int is_order, int gmax, bmat *next, int *err_block) {
    const bmat *A = &L->As;
    int p = A->p;
    int *gid = xmalloc(sizeof(int) * (size_t)(p ? p : 1));
    int ng = level_groups(A, gmax, is_order, gid);
    /* P_I: the groups by their smallest supernode, members ascending, then the rest
     * ascending.  num[I] = group of I or position among the rest; goff[I] = scalar offset
     * of an IS supernode inside its group. */
    int *gnew = xmalloc(sizeof(int) * (size_t)(ng ? ng : 1));
    for (int g = 0; g < ng; ++g) gnew[g] = -1;
    int seen = 0;
    for (int I = 0; I < p; ++I)
        if (gid[I] >= 0 && gnew[gid[I]] < 0) gnew[gid[I]] = seen++;
    for (int I = 0; I < p; ++I)
        if (gid[I] >= 0) gid[I] = gnew[gid[I]];
    free(gnew);
    int *num = xmalloc(sizeof(int) * (size_t)(p ? p : 1));
    int *goff = xmalloc(sizeof(int) * (size_t)(p ? p : 1));
    L->nis = ng;
    L->gptr = xcalloc((size_t)ng + 1, sizeof(int));
    L->nis_sn = 0;
    for (int I = 0; I < p; ++I)
        if (gid[I] >= 0) { L->gptr[gid[I] + 1]++; L->nis_sn++; }
    for (int g = 0; g < ng; ++g) L->gptr[g + 1] += L->gptr[g];
    int nrest = p - L->nis_sn;
    L->is_list = xmalloc(sizeof(int) * (size_t)(L->nis_sn ? L->nis_sn : 1));
    L->rest_list = xmalloc(sizeof(int) * (size_t)(nrest ? nrest : 1));
    L->is_rb = xcalloc((size_t)ng + 1, sizeof(int));
    L->rest_rb = xmalloc(sizeof(int) * ((size_t)nrest + 1));
    int *fill = xmalloc(sizeof(int) * (size_t)(ng ? ng : 1));
    for (int g = 0; g < ng; ++g) fill[g] = L->gptr[g];
    int b = 0;
    L->rest_rb[0] = 0;
    for (int I = 0; I < p; ++I) {
        int m = bm_rs(A, I);
        if (gid[I] >= 0) {
            int g = gid[I];
            L->is_list[fill[g]++] = I;
            num[I] = g;
            goff[I] = L->is_rb[g + 1];
            L->is_rb[g + 1] += m;
        } else { L->rest_list[b] = I; num[I] = b; L->rest_rb[b + 1] = L->rest_rb[b] + m; b++; }
    }
    free(fill);
    for (int g = 0; g < ng; ++g) L->is_rb[g + 1] += L->is_rb[g];
    L->n_is = L->is_rb[ng];
    L->is_rows = xmalloc(sizeof(int) * ((size_t)L->n_is + 1));
    L->rest_rows = xmalloc(sizeof(int) * ((size_t)(L->n - L->n_is) + 1));
    for (int g = 0; g < ng; ++g)
        for (int a = L->gptr[g]; a < L->gptr[g + 1]; ++a) {
            int I = L->is_list[a];
            for (int r = 0; r < bm_rs(A, I); ++r) L->is_rows[L->is_rb[g] + goff[I] + r] = A->rb[I] + r;
        }
    for (int j = 0; j < nrest; ++j) {
        int J = L->rest_list[j];
        for (int r = 0; r < bm_rs(A, J); ++r) L->rest_rows[L->rest_rb[j] + r] = A->rb[J] + r;
    }

    /* pivot blocks: every D_i assembled dense from the blocks among its members, then GEPP */
    L->dlu_off = xmalloc(sizeof(int64_t) * ((size_t)ng + 1));
    L->dlu_off[0] = 0;
    for (int g = 0; g < ng; ++g) {
        int m = L->is_rb[g + 1] - L->is_rb[g];
        L->dlu_off[g + 1] = L->dlu_off[g] + (int64_t)m * m;
    }
    L->dlu = xcalloc((size_t)L->dlu_off[ng] + 1, sizeof(double));
    L->dpiv = xcalloc((size_t)L->n_is + 1, sizeof(int));
    for (int g = 0; g < ng; ++g) {
        int m = L->is_rb[g + 1] - L->is_rb[g];
        double *d = L->dlu + L->dlu_off[g];
        for (int a = L->gptr[g]; a < L->gptr[g + 1]; ++a) {
            int I = L->is_list[a], mI = bm_rs(A, I);
            for (int64_t k = A->rp[I]; k < A->rp[I + 1]; ++k) {
                int J = A->ci[k], nJ = bm_cs(A, J);
                if (gid[J] != g) continue;
                const double *blk = bm_blk(A, k);
                for (int r = 0; r < mI; ++r)
                    for (int c = 0; c < nJ; ++c) d[(goff[I] + r) * m + goff[J] + c] = blk[r * nJ + c];
            }
        }
        if (gepp(m, d, L->dpiv + L->is_rb[g]) != ORC_OK) {
            *err_block = L->is_list[L->gptr[g]];
            free(gid); free(num); free(goff);
            return ORC_ERR_SINGULAR;
        }
    }

    /* G = L^{-1} P F, group by group; a block is the group's rows against one remaining
     * supernode, stacked from the members' blocks */
    bm_init(&L->G, ng, L->is_rb, nrest, L->rest_rb);
    double *tmp = NULL, *colv = NULL;
    int64_t tcap = 0;
    int *cols = xmalloc(sizeof(int) * (size_t)(A->nb ? A->nb : 1));
    for (int g = 0; g < ng; ++g) {
        int m = L->is_rb[g + 1] - L->is_rb[g];
        const double *d = L->dlu + L->dlu_off[g];
        const int *pv = L->dpiv + L->is_rb[g];
        colv = xrealloc(colv, sizeof(double) * (size_t)m);
        int nc = 0;
        for (int a = L->gptr[g]; a < L->gptr[g + 1]; ++a) {
            int I = L->is_list[a];
            for (int64_t k = A->rp[I]; k < A->rp[I + 1]; ++k)
                if (gid[A->ci[k]] < 0) cols[nc++] = num[A->ci[k]];
        }
        qsort(cols, (size_t)nc, sizeof(int), cmp_int);
        for (int e = 0; e < nc; ++e) {
            if (e > 0 && cols[e] == cols[e - 1]) continue;
            int K = cols[e], J = L->rest_list[K], nJ = bm_cs(A, J);
            if ((int64_t)m * nJ > tcap) { tcap = (int64_t)m * nJ; tmp = xrealloc(tmp, sizeof(double) * tcap); }
            memset(tmp, 0, sizeof(double) * (size_t)m * nJ);
            for (int a = L->gptr[g]; a < L->gptr[g + 1]; ++a) {
                int I = L->is_list[a], mI = bm_rs(A, I);
                int64_t k = bm_find(A, I, J);
                if (k < 0) continue;
                const double *fb = bm_blk(A, k);
                for (int r = 0; r < mI; ++r)
                    for (int c = 0; c < nJ; ++c) tmp[(goff[I] + r) * nJ + c] = fb[r * nJ + c];
            }
            for (int c = 0; c < nJ; ++c) {
                for (int r = 0; r < m; ++r) colv[r] = tmp[r * nJ + c];
                lu_fwd(m, d, pv, colv);
                for (int r = 0; r < m; ++r) tmp[r * nJ + c] = colv[r];
            }
            if (!drop_block(m, nJ, tmp, t)) bm_push(&L->G, K, tmp);
        }
        bm_end_row(&L->G);
    }
    /* W = E U^{-1}, row by row of the remaining supernodes; a block is one remaining
     * supernode's rows against a whole group, its members' blocks side by side */
    bm_init(&L->W, nrest, L->rest_rb, ng, L->is_rb);
    for (int j = 0; j < nrest; ++j) {
        int J = L->rest_list[j], m = bm_rs(A, J);
        int nc = 0;
        for (int64_t k = A->rp[J]; k < A->rp[J + 1]; ++k)
            if (gid[A->ci[k]] >= 0) cols[nc++] = gid[A->ci[k]];
        qsort(cols, (size_t)nc, sizeof(int), cmp_int);
        for (int e = 0; e < nc; ++e) {
            if (e > 0 && cols[e] == cols[e - 1]) continue;
            int g = cols[e], mg = L->is_rb[g + 1] - L->is_rb[g];
            if ((int64_t)m * mg > tcap) { tcap = (int64_t)m * mg; tmp = xrealloc(tmp, sizeof(double) * tcap); }
            memset(tmp, 0, sizeof(double) * (size_t)m * mg);
            for (int64_t k = A->rp[J]; k < A->rp[J + 1]; ++k) {
                int I = A->ci[k];
                if (gid[I] != g) continue;
                int nI = bm_cs(A, I);
                const double *eb = bm_blk(A, k);
                for (int r = 0; r < m; ++r)
                    for (int c = 0; c < nI; ++c) tmp[r * mg + goff[I] + c] = eb[r * nI + c];
            }
            const double *d = L->dlu + L->dlu_off[g];
            for (int r = 0; r < m; ++r) row_solve_u(mg, d, tmp + r * mg);
            if (!drop_block(m, mg, tmp, t)) bm_push(&L->W, g, tmp);
        }
        bm_end_row(&L->W);
    }
    free(cols);
    /* Schur complement A_{l+1} = C - W G (Eq. schurl), row by row */
    bm_init(next, nrest, L->rest_rb, nrest, L->rest_rb);
    int64_t *slot = xmalloc(sizeof(int64_t) * (size_t)(nrest ? nrest : 1));
    for (int j = 0; j < nrest; ++j) slot[j] = -1;
    int *keys = xmalloc(sizeof(int) * (size_t)(nrest ? nrest : 1));
    double *acc = NULL;
    int64_t acc_cap = 0;
    for (int j = 0; j < nrest; ++j) {
        int J = L->rest_list[j], m = bm_rs(A, J);
        int nk = 0;
        int64_t used = 0;
        /* C row */
        for (int64_t k = A->rp[J]; k < A->rp[J + 1]; ++k) {
            int K = A->ci[k];
            if (gid[K] >= 0) continue;
            int nK = bm_cs(A, K);
            if (used + (int64_t)m * nK > acc_cap) { acc_cap = 2 * (used + (int64_t)m * nK); acc = xrealloc(acc, sizeof(double) * acc_cap); }
            slot[num[K]] = used;
            keys[nk++] = num[K];
            memcpy(acc + used, bm_blk(A, k), sizeof(double) * m * nK);
            used += (int64_t)m * nK;
        }
        /* subtract W_ji G_i. for every kept W block, ascending i */
        for (int64_t w = L->W.rp[j]; w < L->W.rp[j + 1]; ++w) {
            int i = L->W.ci[w];
            int mi = L->is_rb[i + 1] - L->is_rb[i];
            const double *wb = bm_blk(&L->W, w);
            for (int64_t g = L->G.rp[i]; g < L->G.rp[i + 1]; ++g) {
                int K = L->G.ci[g];
                int nK = L->rest_rb[K + 1] - L->rest_rb[K];
                if (slot[K] < 0) {
                    if (used + (int64_t)m * nK > acc_cap) { acc_cap = 2 * (used + (int64_t)m * nK); acc = xrealloc(acc, sizeof(double) * acc_cap); }
                    slot[K] = used;
                    keys[nk++] = K;
                    memset(acc + used, 0, sizeof(double) * m * nK);
                    used += (int64_t)m * nK;
                }
                double *s = acc + slot[K];
                const double *gb = bm_blk(&L->G, g);
                for (int r = 0; r < m; ++r)
                    for (int c = 0; c < nK; ++c)
                        for (int q = 0; q < mi; ++q)
                            s[r * nK + c] = s[r * nK + c] - wb[r * mi + q] * gb[q * nK + c];
            }
        }
        qsort(keys, nk, sizeof(int), cmp_int);
        for (int t2 = 0; t2 < nk; ++t2) {
            int K = keys[t2];
            int nK = L->rest_rb[K + 1] - L->rest_rb[K];
            const double *s = acc + slot[K];
            if (K == j || !drop_schur || !drop_block(m, nK, s, t)) bm_push(next, K, s);
            slot[K] = -1;
        }
        bm_end_row(next);
    }
    free(acc); free(slot); free(keys); free(tmp); free(colv);
    free(gid); free(num); free(goff);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Last level: block ILUT, IKJ order (Sec. 3, Alg. 3; R5)                    */
/* ------------------------------------------------------------------------- */
static int last_ilut(orc_t *h, double t, int *err_block) {
    const bmat *A = &h->last;
    int p = A->p;
    bm_init(&h->L, p, A->rb, p, A->cb);
    bm_init(&h->U, p, A->rb, p, A->cb);
    h->dl_off = xmalloc(sizeof(int64_t) * ((size_t)p + 1));
    h->dl_off[0] = 0;
    for (int i = 0; i < p; ++i) h->dl_off[i + 1] = h->dl_off[i] + (int64_t)bm_rs(A, i) * bm_rs(A, i);
    h->dl = xcalloc((size_t)h->dl_off[p] + 1, sizeof(double));
    h->dl_piv = xcalloc((size_t)A->rb[p] + 1, sizeof(int));
    int64_t *slot = xmalloc(sizeof(int64_t) * (size_t)(p ? p : 1));
    for (int j = 0; j < p; ++j) slot[j] = -1;
    int *keys = xmalloc(sizeof(int) * (size_t)(p ? p : 1));
    char *state = xcalloc((size_t)p + 1, 1); /* 0 absent/pending, 1 eliminated, 2 dropped */
    double *acc = NULL;
    int64_t acc_cap = 0;
    for (int i = 0; i < p; ++i) {
        int m = bm_rs(A, i);
        int nk = 0;
        int64_t used = 0;
        for (int64_t k = A->rp[i]; k < A->rp[i + 1]; ++k) {
            int K = A->ci[k], nK = bm_cs(A, K);
            if (used + (int64_t)m * nK > acc_cap) { acc_cap = 2 * (used + (int64_t)m * nK); acc = xrealloc(acc, sizeof(double) * acc_cap); }
            slot[K] = used; keys[nk++] = K; state[K] = 0;
            memcpy(acc + used, bm_blk(A, k), sizeof(double) * m * nK);
            used += (int64_t)m * nK;
        }
        int last_k = -1;
        for (;;) {
            /* smallest pending column left of the diagonal */
            int k = -1;
            for (int t2 = 0; t2 < nk; ++t2) {
                int K = keys[t2];
                if (K < i && K > last_k && state[K] == 0 && (k < 0 || K < k)) k = K;
            }
            if (k < 0) break;
            last_k = k;
            int mk = bm_rs(A, k);
            double *wk = acc + slot[k];
            const double *dk = h->dl + h->dl_off[k];
            const int *pk = h->dl_piv + A->rb[k];
            for (int r = 0; r < m; ++r) { row_solve_u(mk, dk, wk + r * mk); row_solve_lp(mk, dk, pk, wk + r * mk); }
            if (drop_block(m, mk, wk, t)) { state[k] = 2; continue; }
            state[k] = 1;
            for (int64_t u = h->U.rp[k]; u < h->U.rp[k + 1]; ++u) {
                int J = h->U.ci[u], nJ = bm_cs(A, J);
                if (slot[J] < 0) {
                    if (used + (int64_t)m * nJ > acc_cap) {
                        acc_cap = 2 * (used + (int64_t)m * nJ);
                        acc = xrealloc(acc, sizeof(double) * acc_cap);
                        wk = acc + slot[k];
                    }
                    slot[J] = used; keys[nk++] = J; state[J] = 0;
                    memset(acc + used, 0, sizeof(double) * m * nJ);
                    used += (int64_t)m * nJ;
                }
                double *wj = acc + slot[J];
                const double *ub = bm_blk(&h->U, u);
                for (int r = 0; r < m; ++r)
                    for (int c = 0; c < nJ; ++c)
                        for (int q = 0; q < mk; ++q)
                            wj[r * nJ + c] = wj[r * nJ + c] - wk[r * mk + q] * ub[q * nJ + c];
            }
        }
        qsort(keys, nk, sizeof(int), cmp_int);
        if (slot[i] < 0) { *err_block = i; free(acc); free(slot); free(keys); free(state); return ORC_ERR_SINGULAR; }
        for (int t2 = 0; t2 < nk; ++t2) {
            int K = keys[t2];
            if (K < i && state[K] == 1) bm_push(&h->L, K, acc + slot[K]);
        }
        bm_end_row(&h->L);
        double *d = h->dl + h->dl_off[i];
        memcpy(d, acc + slot[i], sizeof(double) * m * m);
        if (gepp(m, d, h->dl_piv + A->rb[i]) != ORC_OK) {
            *err_block = i; free(acc); free(slot); free(keys); free(state); return ORC_ERR_SINGULAR;
        }
        for (int t2 = 0; t2 < nk; ++t2) {
            int K = keys[t2];
            if (K > i && !drop_block(m, bm_cs(A, K), acc + slot[K], t)) bm_push(&h->U, K, acc + slot[K]);
        }
        bm_end_row(&h->U);
        for (int t2 = 0; t2 < nk; ++t2) { slot[keys[t2]] = -1; state[keys[t2]] = 0; }
    }
    free(acc); free(slot); free(keys); free(state);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Construction                                                              */
/* ------------------------------------------------------------------------- */
void orc_free(orc_t *h);

orc_t *orc_build(int n, const int64_t *rowptr, const int32_t *col, const double *val,
                 const int32_t *perm, const int32_t *bptr, int p,
                 int levels, const double *droptol, int drop_schur, int is_order, int group_rows) {
    orc_t *h = xcalloc(1, sizeof(orc_t));
    h->n = n; h->p = p;
    h->err_level = -1; h->err_block = -1;
    h->perm = xmalloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    h->bptr = xmalloc(sizeof(int32_t) * ((size_t)p + 1));
    memcpy(h->perm, perm, sizeof(int32_t) * (size_t)n);
    memcpy(h->bptr, bptr, sizeof(int32_t) * ((size_t)p + 1));
    if (levels < 0 || levels > 16 || group_rows < 0) { h->status = ORC_ERR_ARG; return h; }
    h->lev = xcalloc((size_t)levels + 1, sizeof(olevel));
    bmat cur;
    build_vbcsr(n, rowptr, col, val, perm, bptr, p, &cur);
    h->nlev = 0;
    for (int l = 0; l < levels; ++l) {
        if (cur.p == 0) break;
        olevel *L = &h->lev[l];
        L->A = cur;
        L->p = cur.p; L->n = cur.rb[cur.p];
        level_scale(L);
        bmat next;
        int eb = -1;
        int st = level_factor(L, droptol[l], drop_schur, is_order, group_rows, &next, &eb);
        h->nlev = l + 1;
        if (st != ORC_OK) { h->status = st; h->err_level = l; h->err_block = eb; memset(&h->last, 0, sizeof(bmat)); return h; }
        cur = next;
        if (L->nis == 0) break; /* nothing eliminated: stop reducing */
    }
    h->last = cur;
    int eb = -1;
    int st = last_ilut(h, droptol[levels], &eb);
    if (st != ORC_OK) { h->status = st; h->err_level = h->nlev; h->err_block = eb; }
    return h;
}

static void free_level(olevel *L) {
    bm_free(&L->A); bm_free(&L->As); bm_free(&L->G); bm_free(&L->W);
    free(L->s1); free(L->s2); free(L->is_list); free(L->rest_list); free(L->gptr);
    free(L->is_rows); free(L->rest_rows);
    free(L->dlu); free(L->dlu_off); free(L->dpiv); free(L->is_rb); free(L->rest_rb);
}

void orc_free(orc_t *h) {
    if (!h) return;
    for (int l = 0; l < h->nlev; ++l) free_level(&h->lev[l]);
    free(h->lev);
    if (h->last.rb) bm_free(&h->last);
    if (h->L.rb) bm_free(&h->L);
    if (h->U.rb) bm_free(&h->U);
    free(h->dl); free(h->dl_off); free(h->dl_piv); free(h->perm); free(h->bptr);
    free(h);
}

int orc_status(const orc_t *h, int *err_level, int *err_block) {
    if (err_level) *err_level = h->err_level;
    if (err_block) *err_block = h->err_block;
    return h->status;
}

/* ------------------------------------------------------------------------- */
/* Preconditioner application (Alg. 2 with the permutations and scalings)     */
/* ------------------------------------------------------------------------- */

/* last level: x = U_S^{-1} L_S^{-1} g (in place) */
static void last_solve(const orc_t *h, double *x) {
    const bmat *A = &h->last;
    int p = A->p;
    for (int i = 0; i < p; ++i) {
        int m = bm_rs(A, i);
        double *xi = x + A->rb[i];
        for (int64_t k = h->L.rp[i]; k < h->L.rp[i + 1]; ++k) {
            int K = h->L.ci[k], nK = bm_cs(A, K);
            const double *b = bm_blk(&h->L, k);
            const double *xk = x + A->rb[K];
            for (int r = 0; r < m; ++r)
                for (int q = 0; q < nK; ++q) xi[r] = xi[r] - b[r * nK + q] * xk[q];
        }
    }
    for (int i = p - 1; i >= 0; --i) {
        int m = bm_rs(A, i);
        double *xi = x + A->rb[i];
        for (int64_t k = h->U.rp[i]; k < h->U.rp[i + 1]; ++k) {
            int K = h->U.ci[k], nK = bm_cs(A, K);
            const double *b = bm_blk(&h->U, k);
            const double *xk = x + A->rb[K];
            for (int r = 0; r < m; ++r)
                for (int q = 0; q < nK; ++q) xi[r] = xi[r] - b[r * nK + q] * xk[q];
        }
        const double *d = h->dl + h->dl_off[i];
        lu_fwd(m, d, h->dl_piv + A->rb[i], xi);
        lu_bwd(m, d, xi);
    }
}

/* x_l = A_l^{-1} b_l approximately, both in the numbering of level l */
static void level_solve(const orc_t *h, int l, const double *b, double *x) {
    if (l == h->nlev) {
        int n = h->last.rb[h->last.p];
        memcpy(x, b, sizeof(double) * (size_t)n);
        last_solve(h, x);
        return;
    }
    const olevel *L = &h->lev[l];
    int nrest = L->p - L->nis_sn;
    int nr = L->rest_rb[nrest];
    double *y = xmalloc(sizeof(double) * ((size_t)L->n_is + 1));
    double *g = xmalloc(sizeof(double) * ((size_t)nr + 1));
    double *z = xmalloc(sizeof(double) * ((size_t)nr + 1));
    /* f = (S1 b) restricted to the independent set; y = L^{-1} P f per group */
    for (int i = 0; i < L->nis; ++i) {
        int m = L->is_rb[i + 1] - L->is_rb[i];
        const int *rows = L->is_rows + L->is_rb[i];
        double *yi = y + L->is_rb[i];
        for (int r = 0; r < m; ++r) yi[r] = L->s1[rows[r]] * b[rows[r]];
        lu_fwd(m, L->dlu + L->dlu_off[i], L->dpiv + L->is_rb[i], yi);
    }
    /* g' = S1 g - W y */
    for (int j = 0; j < nrest; ++j) {
        int m = L->rest_rb[j + 1] - L->rest_rb[j];
        const int *rows = L->rest_rows + L->rest_rb[j];
        double *gj = g + L->rest_rb[j];
        for (int r = 0; r < m; ++r) gj[r] = L->s1[rows[r]] * b[rows[r]];
        for (int64_t k = L->W.rp[j]; k < L->W.rp[j + 1]; ++k) {
            int i = L->W.ci[k];
            int mi = L->is_rb[i + 1] - L->is_rb[i];
            const double *wb = bm_blk(&L->W, k);
            for (int r = 0; r < m; ++r)
                for (int q = 0; q < mi; ++q) gj[r] = gj[r] - wb[r * mi + q] * y[L->is_rb[i] + q];
        }
    }
    level_solve(h, l + 1, g, z);
    /* u = U^{-1} (y - G z) per group; x = S2 P_I^T (u, z) */
    for (int i = 0; i < L->nis; ++i) {
        int m = L->is_rb[i + 1] - L->is_rb[i];
        const int *rows = L->is_rows + L->is_rb[i];
        double *yi = y + L->is_rb[i];
        for (int64_t k = L->G.rp[i]; k < L->G.rp[i + 1]; ++k) {
            int K = L->G.ci[k];
            int nK = L->rest_rb[K + 1] - L->rest_rb[K];
            const double *gb = bm_blk(&L->G, k);
            for (int r = 0; r < m; ++r)
                for (int q = 0; q < nK; ++q) yi[r] = yi[r] - gb[r * nK + q] * z[L->rest_rb[K] + q];
        }
        lu_bwd(m, L->dlu + L->dlu_off[i], yi);
        for (int r = 0; r < m; ++r) x[rows[r]] = L->s2[rows[r]] * yi[r];
    }
    for (int j = 0; j < nrest; ++j) {
        int m = L->rest_rb[j + 1] - L->rest_rb[j];
        const int *rows = L->rest_rows + L->rest_rb[j];
        for (int r = 0; r < m; ++r) x[rows[r]] = L->s2[rows[r]] * z[L->rest_rb[j] + r];
    }
    free(y); free(g); free(z);
}

/* y = M^{-1} x in the original numbering: x_1 = P_B x, solve, y = P_B^T x_1 */
int orc_apply(const orc_t *h, const double *x, double *y) {
    if (h->status != ORC_OK) return ORC_ERR_STATE;
    int n = h->n;
    double *b1 = xmalloc(sizeof(double) * ((size_t)n + 1));
    double *x1 = xmalloc(sizeof(double) * ((size_t)n + 1));
    for (int k = 0; k < n; ++k) b1[k] = x[h->perm[k]];
    level_solve(h, 0, b1, x1);
    for (int k = 0; k < n; ++k) y[h->perm[k]] = x1[k];
    free(b1); free(x1);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Right-preconditioned FGMRES(m) (Sec. 4.1; Saad 1993), modified Gram-Schmidt */
/* ------------------------------------------------------------------------- */
static void csr_mv(int n, const int64_t *rp, const int32_t *ci, const double *v, const double *x, double *y) {
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s = s + v[k] * x[ci[k]];
        y[i] = s;
    }
}
static double dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s = s + a[i] * b[i];
    return s;
}

/* Solves A x = b.  x holds the initial guess on entry.  Stops when the true residual
 * ||b - A x|| <= tol ||b|| or after maxit inner iterations.  hist (optional, length
 * maxit + 1) receives the Arnoldi residual estimate after every iteration, relative to
 * ||b||.  If h is NULL the preconditioner is the identity. */
int orc_fgmres(const orc_t *h, int n, const int64_t *rp, const int32_t *ci, const double *av,
               const double *b, double *x, double tol, int m, int maxit,
               int *iters, double *relres, double *hist) {
    if (h && h->status != ORC_OK) return ORC_ERR_STATE;
    if (m < 1 || maxit < 0 || n < 0) return ORC_ERR_ARG;
    double *V = xmalloc(sizeof(double) * (size_t)(m + 1) * (size_t)(n ? n : 1));
    double *Z = xmalloc(sizeof(double) * (size_t)m * (size_t)(n ? n : 1));
    double *H = xcalloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = xmalloc(sizeof(double) * m), *sn = xmalloc(sizeof(double) * m);
    double *gv = xmalloc(sizeof(double) * (m + 1)), *yv = xmalloc(sizeof(double) * (m + 1));
    double *w = xmalloc(sizeof(double) * (size_t)(n ? n : 1));
    double bn = sqrt(dot(n, b, b));
    int it = 0, status = ORC_NOT_CONVERGED;
    double rel = 0.0;
    if (bn == 0.0) { for (int i = 0; i < n; ++i) x[i] = 0.0; *iters = 0; *relres = 0.0; status = ORC_OK; goto done; }
    for (;;) {
        csr_mv(n, rp, ci, av, x, w);
        for (int i = 0; i < n; ++i) V[i] = b[i] - w[i];
        double beta = sqrt(dot(n, V, V));
        rel = beta / bn;
        if (rel <= tol) { status = ORC_OK; break; }
        if (it >= maxit) break;
        for (int i = 0; i < n; ++i) V[i] = V[i] / beta;
        for (int k = 0; k <= m; ++k) gv[k] = 0.0;
        gv[0] = beta;
        int j = 0;
        for (; j < m && it < maxit; ++j) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
            if (h) orc_apply(h, vj, zj); else memcpy(zj, vj, sizeof(double) * n);
            csr_mv(n, rp, ci, av, zj, vn);
            for (int k = 0; k <= j; ++k) {
                double hk = dot(n, vn, V + (size_t)k * n);
                H[k * m + j] = hk;
                for (int i = 0; i < n; ++i) vn[i] = vn[i] - hk * V[(size_t)k * n + i];
            }
            double hn = sqrt(dot(n, vn, vn));
            H[(j + 1) * m + j] = hn;
            if (hn > 0.0) for (int i = 0; i < n; ++i) vn[i] = vn[i] / hn;
            for (int k = 0; k < j; ++k) {
                double a = H[k * m + j], c = H[(k + 1) * m + j];
                H[k * m + j] = cs[k] * a + sn[k] * c;
                H[(k + 1) * m + j] = -sn[k] * a + cs[k] * c;
            }
            double a = H[j * m + j], c = H[(j + 1) * m + j];
            double r = sqrt(a * a + c * c);
            cs[j] = r > 0.0 ? a / r : 1.0;
            sn[j] = r > 0.0 ? c / r : 0.0;
            H[j * m + j] = r;
            H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            it++;
            if (hist) hist[it] = fabs(gv[j + 1]) / bn;
            if (fabs(gv[j + 1]) <= tol * bn || hn == 0.0) { j++; break; }
        }
        /* x = x + Z y with H(0:j,0:j) y = g */
        for (int k = j - 1; k >= 0; --k) {
            double s = gv[k];
            for (int q = k + 1; q < j; ++q) s = s - H[k * m + q] * yv[q];
            yv[k] = s / H[k * m + k];
        }
        for (int k = 0; k < j; ++k)
            for (int i = 0; i < n; ++i) x[i] = x[i] + yv[k] * Z[(size_t)k * n + i];
    }
    *iters = it;
    *relres = rel;
done:
    if (hist) hist[0] = 1.0;
    free(V); free(Z); free(H); free(cs); free(sn); free(gv); free(yv); free(w);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Inspection (tests compare these against the GPU library)                  */
/* ------------------------------------------------------------------------- */
enum { W_A = 0, W_AS = 1, W_G = 2, W_W = 3, W_D = 4, W_LAST = 5, W_L = 6, W_U = 7, W_DL = 8 };

int orc_nlevels(const orc_t *h) { return h->nlev; }

/* info: p, n, groups, n_is, supernodes in the groups */
int orc_level_info(const orc_t *h, int l, int32_t *info) {
    if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    const olevel *L = &h->lev[l];
    info[0] = L->p; info[1] = L->n; info[2] = L->nis; info[3] = L->n_is; info[4] = L->nis_sn;
    return ORC_OK;
}
/* the supernodes of the groups, group after group (info[4] entries) */
int orc_level_is(const orc_t *h, int l, int32_t *is_list) {
    if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    memcpy(is_list, h->lev[l].is_list, sizeof(int) * (size_t)h->lev[l].nis_sn);
    return ORC_OK;
}
/* group pointers into the list above (info[2] + 1 entries) */
int orc_level_groups(const orc_t *h, int l, int32_t *gptr) {
    if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    memcpy(gptr, h->lev[l].gptr, sizeof(int) * ((size_t)h->lev[l].nis + 1));
    return ORC_OK;
}
int orc_level_scaling(const orc_t *h, int l, double *s1, double *s2) {
    if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    memcpy(s1, h->lev[l].s1, sizeof(double) * (size_t)h->lev[l].n);
    memcpy(s2, h->lev[l].s2, sizeof(double) * (size_t)h->lev[l].n);
    return ORC_OK;
}

static const bmat *pick(const orc_t *h, int which, int l) {
    if (which == W_LAST) return &h->last;
    if (which == W_L) return &h->L;
    if (which == W_U) return &h->U;
    if (l < 0 || l >= h->nlev) return NULL;
    const olevel *L = &h->lev[l];
    switch (which) {
    case W_A: return &L->A;
    case W_AS: return &L->As;
    case W_G: return &L->G;
    case W_W: return &L->W;
    default: return NULL;
    }
}

/* dims: p_rows, p_cols, nb, nvals */
int orc_matrix_dims(const orc_t *h, int which, int l, int64_t *dims) {
    if (which == W_D || which == W_DL) {
        int nb;
        int64_t nv;
        if (which == W_D) { if (l < 0 || l >= h->nlev) return ORC_ERR_ARG; nb = h->lev[l].nis; nv = h->lev[l].dlu_off[nb]; }
        else { nb = h->last.p; nv = h->dl_off[nb]; }
        dims[0] = nb; dims[1] = nb; dims[2] = nb; dims[3] = nv;
        return ORC_OK;
    }
    const bmat *a = pick(h, which, l);
    if (!a || !a->rb) return ORC_ERR_ARG;
    dims[0] = a->p; dims[1] = a->q; dims[2] = a->nb; dims[3] = a->vo[a->nb];
    return ORC_OK;
}

/* block sparse export: rb[p+1], cb[q+1], rowptr[p+1], colidx[nb], vals[nvals];
 * for W_D / W_DL the pivot blocks as a block diagonal, pivots in piv (scalar length) */
int orc_matrix_get(const orc_t *h, int which, int l, int32_t *rb, int32_t *cb, int64_t *rowptr,
                   int32_t *colidx, double *vals, int32_t *piv) {
    if (which == W_D || which == W_DL) {
        int nb;
        const int *srb;
        const double *v;
        const int64_t *off;
        const int *pv;
        if (which == W_D) {
            if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
            nb = h->lev[l].nis; srb = h->lev[l].is_rb; v = h->lev[l].dlu; off = h->lev[l].dlu_off; pv = h->lev[l].dpiv;
        } else {
            nb = h->last.p; srb = h->last.rb; v = h->dl; off = h->dl_off; pv = h->dl_piv;
        }
        for (int i = 0; i <= nb; ++i) { rb[i] = srb[i]; cb[i] = srb[i]; rowptr[i] = i; }
        for (int i = 0; i < nb; ++i) colidx[i] = i;
        memcpy(vals, v, sizeof(double) * (size_t)off[nb]);
        if (piv) memcpy(piv, pv, sizeof(int) * (size_t)srb[nb]);
        return ORC_OK;
    }
    const bmat *a = pick(h, which, l);
    if (!a || !a->rb) return ORC_ERR_ARG;
    memcpy(rb, a->rb, sizeof(int) * ((size_t)a->p + 1));
    memcpy(cb, a->cb, sizeof(int) * ((size_t)a->q + 1));
    memcpy(rowptr, a->rp, sizeof(int64_t) * ((size_t)a->p + 1));
    memcpy(colidx, a->ci, sizeof(int) * (size_t)a->nb);
    memcpy(vals, a->v, sizeof(double) * (size_t)a->vo[a->nb]);
    return ORC_OK;
}

/* nnz(preconditioner) counted as stored block entries of all factors (Mem numerator) */
int64_t orc_factor_nnz(const orc_t *h) {
    int64_t s = 0;
    for (int l = 0; l < h->nlev; ++l) {
        const olevel *L = &h->lev[l];
        s += L->dlu_off[L->nis] + L->G.vo[L->G.nb] + L->W.vo[L->W.nb];
    }
    if (h->L.rb) s += h->L.vo[h->L.nb] + h->U.vo[h->U.nb] + h->dl_off[h->last.p];
    return s;
}
