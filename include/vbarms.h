/*
 * vbarms.h -- C ABI of the MI355X VBARMS library (libvbarms.so).
 *
 * VBARMS is the variable-block algebraic recursive multilevel ILU preconditioner of
 * Carpentieri, Liao, Sosonkina and Bonfiglioli, "Using the VBARMS method in parallel
 * computing" (arXiv:1508.02219).  This library runs the method's hot path on one
 * gfx950 GPU:
 *
 *   vbarms_compress  angle-based compression of a CSR matrix into variable blocks
 *                    (Sec. 2.1) and the permuted variable-block matrix (Eq. blockperm)
 *   vbarms_factor    per level: scaling (Sec. 3 Step 2), block independent set on the
 *                    quotient graph (Step 3), partial block factorization with
 *                    threshold dropping (Step 4, Eq. vbarms, Eq. schurl); block ILUT on
 *                    the last Schur complement (Sec. 3, Alg. 3)
 *   vbarms_apply     the multilevel solve (Alg. 2) with the inverse permutations
 *   vbarms_spmv      y = A x with the compressed matrix
 *   vbarms_solve     right-preconditioned FGMRES(m) (Sec. 4.1)
 *
 * Conventions
 *  - Every pointer documented as DEVICE must point to memory allocated on the handle's
 *    device (hipMalloc or a torch CUDA tensor); HOST pointers are ordinary host memory.
 *  - The caller owns every buffer passed in; the library never keeps a caller pointer
 *    after the call returns (vbarms_compress copies what it needs).
 *  - The handle owns the compressed matrix, all factors and all workspace until
 *    vbarms_destroy.
 *  - Work is enqueued on the stream given to vbarms_create.  Calls that return host
 *    data (statistics, solver info, exports) synchronize that stream.
 *  - Indices: rows, columns and blocks are int32; offsets into value arrays are int64.
 *  - Every call returns VBARMS_OK (0) on success, VBARMS_NOT_CONVERGED (1) when a solve
 *    ran to maxit without meeting tol (its result and info are still valid), or a
 *    negative error code; vbarms_last_error() then describes the failure.  No C++
 *    exception crosses this interface.
 *  - A handle is not thread safe; different handles may be used concurrently.
 */
#ifndef VBARMS_H
#define VBARMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VBARMS_OK 0
#define VBARMS_NOT_CONVERGED 1
#define VBARMS_ERR_ARG (-1)      /* invalid argument (sizes, tau outside (0,1], NULL) */
#define VBARMS_ERR_HIP (-2)      /* a HIP runtime call failed */
#define VBARMS_ERR_OOM (-3)      /* device allocation or a documented capacity exceeded */
#define VBARMS_ERR_SINGULAR (-4) /* a pivot block is exactly singular (GEPP met a zero column) */
#define VBARMS_ERR_NAN (-5)      /* NaN or Inf in the input matrix or right-hand side */
#define VBARMS_ERR_STATE (-6)    /* call out of order (e.g. apply before factor) */

#define VBARMS_MAX_BLOCK 32      /* largest variable block the kernels accept */
#define VBARMS_MAX_LEVELS 16

/* precision of the factors (the Krylov solver is always FP64) */
#define VBARMS_F64 0
#define VBARMS_F32 1

typedef struct vbarms_ctx *vbarms_t;

/* Square sparse matrix in CSR form.  DEVICE pointers: rowptr[n+1] (int64, rowptr[0] = 0),
 * col[nnz] (int32, sorted ascending within each row, no duplicates), val[nnz] (FP64).
 * The stored entries define the pattern (explicit zeros count as entries). */
typedef struct {
    int32_t n;
    int64_t nnz;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
} vbarms_csr;

/* Compression statistics (Sec. 2): av_bd = nnz(A) / (entries of all nonzero blocks),
 * av_bs = n / number of diagonal blocks. */
typedef struct {
    int32_t nblocks;   /* p, number of diagonal blocks (supernodes) */
    int32_t max_block; /* largest block size */
    int64_t nnz_blocks;/* number of nonzero blocks of the permuted matrix */
    double av_bd;
    double av_bs;
} vbarms_cstats;

/* visiting order of the greedy block independent set (Sec. 3, Step 3) */
#define VBARMS_IS_NATURAL 0   /* supernodes in ascending order (Sec. 2, the simple greedy) */
#define VBARMS_IS_WEIGHTED 1  /* descending ||A_II||_F / sum_J ||A_IJ||_F of the scaled level
                                 matrix, ties ascending (Sec. 3, "weighted greedy") */

/* Factorization parameters.  droptol[l] is the threshold t of level l (Sec. 3: a block B
 * of size m x n is dropped when ||B||_F / (m n) < t); droptol[levels] is used by the
 * last-level block ILUT.  drop_schur = 1 also drops small off-diagonal blocks of every
 * Schur complement; 0 keeps them all (the paper's wording for intermediate levels).
 *
 * group_rows selects the groups of the block independent set (Sec. 2 and Sec. 3, Step 3,
 * where the diagonal blocks D_i of D are themselves block sparse): 0 puts one supernode in
 * every group; k in [1, VBARMS_MAX_BLOCK] lets an unmarked supernode v open a group that
 * its unmarked quotient-graph neighbours (A + A^T) join in ascending order whenever the
 * group stays within k rows, after which the members and all their neighbours are marked.
 * A group is one dense pivot block, zero padded where no block is stored, factored exactly
 * by GEPP; a block of L^{-1}F (E U^{-1}) is the group's rows (columns) against one remaining
 * supernode, and the drop rule applies at that size.  The greedy is sequential by
 * definition and runs on the host over a copy of the level's block pattern.
 *
 * Zero-initialize the struct: 0 selects the default of every field. */
typedef struct {
    int32_t levels;                        /* number of Schur reductions (0 = block ILUT only) */
    double droptol[VBARMS_MAX_LEVELS + 1];
    int32_t drop_schur;
    int32_t is_order;                      /* VBARMS_IS_NATURAL or VBARMS_IS_WEIGHTED */
    int32_t precision;                     /* VBARMS_F64 or VBARMS_F32 */
    int32_t group_rows;                    /* 0: one supernode per group; else the row limit */
} vbarms_fparams;

typedef struct {
    int32_t iters;       /* Arnoldi steps taken */
    int32_t restarts;    /* completed restart cycles */
    double true_relres;  /* ||b - A x|| / ||b|| of the returned x */
    int32_t status;      /* same as the return value */
    int32_t fp64_refactor; /* 1 when FP32 factors did not converge within the FP32 step limit and
                              the solve recomputed them in FP64 (see vbarms_set_fp64_fallback) */
} vbarms_sinfo;

/* Phase timings of the last calls, milliseconds of device time on the handle's stream. */
typedef struct {
    double compress_ms, factor_ms, solve_ms;
    double factor_level_ms[VBARMS_MAX_LEVELS];
    double ilut_ms;
    int32_t levels;          /* levels actually factored */
    int32_t last_p;          /* supernodes handed to the last-level ILUT */
    int64_t factor_values;   /* stored values of all factors (Mem = factor_values / nnz(A)) */
    int64_t nnz;             /* nnz(A) */
    int32_t spmv_lanes;      /* lanes per scalar row of the FGMRES product, picked at compression by
                                timing 4, 8, 16 and 32 on the compressed matrix */
    int32_t ilut_waves;      /* dependency-wave launches of the last-level block ILUT */
    int32_t ilut_attempts;   /* runs of the block ILUT: more than 1 when its working room ran out
                                and it started again with more (the handle keeps the larger room) */
    double ilut_result_bytes;/* algorithmic bytes of the block ILUT: its input matrix read once and
                                L, U, the pivot-block LU factors and pivots written once */
    int32_t illcond_blocks;  /* pivot blocks of the last factorization whose pivot ratio (smallest over
                                largest pivot magnitude) fell below the fallback threshold */
    int32_t fp64_fallback;   /* 0: factors in the requested precision; 1: FP32 was requested but an
                                ill-conditioned pivot block sent the factorization to FP64; 2: a
                                solve with FP32 factors stagnated and refactored in FP64 */
} vbarms_fstats;

/* Creates a handle bound to the current HIP device and to `hip_stream` (a hipStream_t,
 * NULL = the null stream).  Returns VBARMS_ERR_HIP if no device is present. */
int vbarms_create(vbarms_t *h, void *hip_stream);
int vbarms_destroy(vbarms_t h);
/* Text of the last error on this handle (never NULL; "" after success). */
const char *vbarms_last_error(vbarms_t h);

/* Angle-based compression (Sec. 2.1): rows i < j share a block when the cosine of their
 * 0/1 patterns is >= tau, comparing each row with the seed of its group only; seeds are
 * taken in ascending row order and empty rows stay alone.  tau must be in (0, 1]; tau = 1
 * groups exactly the rows with identical patterns.  Builds the permuted variable-block
 * matrix inside the handle (Eq. blockperm; every block row carries its diagonal block).
 * Outputs (DEVICE, may be NULL): perm[n] (new position -> original row), bptr[p+1]
 * (scalar offsets of the blocks; caller provides n+1 entries).  st (HOST, may be NULL)
 * receives the statistics.  Errors: ARG (bad tau / n), NAN, OOM (a block row with more
 * than 2048 distinct block columns, or a block larger than VBARMS_MAX_BLOCK). */
int vbarms_compress(vbarms_t h, const vbarms_csr *A, double tau,
                    int32_t *perm, int32_t *bptr, vbarms_cstats *st);

/* Graph-based compression (Sec. 2.2, Alg. 1): rows with identical patterns form the first
 * supernodes; then every supernode, in ascending order of its smallest row, tries the
 * supernodes adjacent to it in the quotient graph of A + A^T (ascending smallest row) and
 * merges with each one while the average block density of the whole ordering -- nnz(A)
 * over the elements of the blocks holding an entry or lying on the diagonal -- stays at
 * least mu; merges beyond VBARMS_MAX_BLOCK rows are skipped.  Blocks follow their smallest
 * row.  mu in (0, 1]; mu = 1 keeps the identical-pattern classes.  The merge loop is
 * sequential by definition and runs on the host over a copy of the pattern.  Outputs and
 * errors as vbarms_compress. */
int vbarms_compress_graph(vbarms_t h, const vbarms_csr *A, double mu,
                          int32_t *perm, int32_t *bptr, vbarms_cstats *st);

/* Uses a given block partition instead of computing one: perm[n], bptr[p+1] are DEVICE
 * arrays with the same meaning as the outputs of vbarms_compress. */
int vbarms_set_partition(vbarms_t h, const vbarms_csr *A, const int32_t *perm,
                         const int32_t *bptr, int32_t p, vbarms_cstats *st);

/* Multilevel factorization of the compressed matrix (Sec. 3, Steps 2-4 repeated, then
 * block ILUT).  Stops early when an independent set is empty or the Schur complement has
 * no rows.  Errors: STATE (no compressed matrix), SINGULAR (exactly singular pivot
 * block; see vbarms_error_location), OOM. */
int vbarms_factor(vbarms_t h, const vbarms_fparams *p);

/* Level and block of the last SINGULAR error (level == levels means the last level). */
int vbarms_error_location(vbarms_t h, int32_t *level, int32_t *block);

/* y = M^{-1} x with the multilevel factors (Alg. 2), DEVICE vectors of length n in the
 * original numbering.  x and y must not overlap.  Errors: STATE before factor. */
int vbarms_apply(vbarms_t h, const double *x, double *y);

/* y = A x with the compressed matrix (original numbering, DEVICE vectors). */
int vbarms_spmv(vbarms_t h, const double *x, double *y);

/* Overrides the lanes per scalar row (4, 8, 16 or 32) that compression picked by timing
 * the product.  Every choice computes the same product up to rounding order.  Errors:
 * STATE before compress, ARG for another value. */
int vbarms_set_spmv_lanes(vbarms_t h, int32_t lanes);

/* y = A x exactly as vbarms_spmv, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  It
 * allocates nothing: the permuted copies of x and y live in a fixed array of
 * 2 * VBARMS_NOALLOC_MAX_N doubles (32 MiB) that the library places on every GPU it runs on
 * and keeps until the process ends.  x, y: DEVICE vectors of length n (original
 * numbering), not overlapping.  Every call on one GPU shares that GPU's array, so calls
 * that overlap in time on one GPU (other handles, other streams) race and must be ordered
 * by the caller.  Errors: STATE (no compressed matrix), ARG (n > VBARMS_NOALLOC_MAX_N or
 * NULL vectors). */
#define VBARMS_NOALLOC_MAX_N (1 << 21)
int vbarms_spmv_noalloc(vbarms_t h, const double *x, double *y);

/* Solves A x = b by FGMRES(restart) preconditioned on the right with M (Sec. 4.1).
 * b, x: DEVICE vectors of length n in the original numbering; x holds the initial guess
 * on entry (zeros for x0 = 0) and the solution on exit.  Stops when the true relative
 * residual ||b - A x|| / ||b|| <= tol, checked at every restart, or after maxit Arnoldi
 * steps (returns VBARMS_NOT_CONVERGED).  info (HOST, may be NULL) is filled either way. */
int vbarms_solve(vbarms_t h, const double *b, double *x, double tol, int32_t restart,
                 int32_t maxit, vbarms_sinfo *info);

/* Safeguards of FP32 factors (mixed precision; FGMRES is FP64 throughout).  With enable != 0
 * (the default):
 *  - a factorization requested in FP32 is redone in FP64 when any pivot block (the
 *    independent-set blocks of every level and the last level's diagonal blocks) has a
 *    pivot ratio min|u_kk| / max|u_kk| below min_pivot_ratio (default 1e-4: at FP32
 *    rounding such a block loses about four more digits than a well-conditioned one);
 *  - a solve with FP32 factors that has not converged after f32_iter_limit Arnoldi steps
 *    (default 100) recomputes the factors in FP64 with the same parameters and continues
 *    FGMRES from its current iterate; vbarms_sinfo.fp64_refactor reports it.
 * The handle's factors stay FP64 afterwards.  Errors: ARG (negative limit, ratio outside
 * [0, 1]). */
int vbarms_set_fp64_fallback(vbarms_t h, int32_t enable, int32_t f32_iter_limit, double min_pivot_ratio);

/* ---------------------------------------------------------------------------------- */
/* Batches of independent systems (not part of the paper's method: a way to run many     */
/* systems of different sizes through the same launches).                               */
/* ---------------------------------------------------------------------------------- */
/* The systems are assembled into one block-diagonal matrix, which is compressed and
 * factored like a single system: rows of different systems share no column, so no block,
 * independent-set decision, Schur update or ILUT row couples two systems, and every system
 * gets exactly the factors it would get alone, while every launch covers all systems.  The
 * solves run FGMRES for every system in lockstep (shared launches, per-system inner
 * products, Hessenberg matrices, convergence and restarts). */
typedef struct vbarms_batch_ctx *vbarms_batch_t;
int vbarms_batch_create(vbarms_batch_t *b, void *hip_stream);
int vbarms_batch_destroy(vbarms_batch_t b);
const char *vbarms_batch_last_error(vbarms_batch_t b);
/* The handle of the combined system (owned by the batch): statistics, timing and the
 * factor exports work on it; its numbering is the concatenation of the systems. */
vbarms_t vbarms_batch_handle(vbarms_batch_t b);
/* systems: HOST array of nsys descriptors whose arrays are DEVICE pointers (as in
 * vbarms_compress; copied, the caller may free them afterwards).  tau and p as in
 * vbarms_compress and vbarms_factor.  Errors: ARG (nsys < 1, more than 2^31 - 1 rows in
 * total), and those of vbarms_compress and vbarms_factor. */
int vbarms_batch_factor(vbarms_batch_t b, int32_t nsys, const vbarms_csr *systems, double tau,
                        const vbarms_fparams *p);
/* off[nsys+1] (HOST): first row of every system in the concatenated numbering. */
int vbarms_batch_offsets(vbarms_batch_t b, int64_t *off);
/* Solves A_s x = b for every system s and every right-hand side r < nrhs.  B, X: DEVICE,
 * nrhs columns of length N = total rows, column r at B + r N, system s's rows at
 * [off_s, off_{s+1}) of a column; X holds the initial guesses on entry.  Per system and
 * column: stops at a true relative residual <= tol or after maxit Arnoldi steps.
 * info (HOST, may be NULL): nrhs * nsys entries, column r's system s at r * nsys + s.
 * Returns VBARMS_NOT_CONVERGED if any system missed tol. */
int vbarms_batch_solve(vbarms_batch_t b, const double *B, double *X, int32_t nrhs, double tol, int32_t restart,
                       int32_t maxit, vbarms_sinfo *info);

/* Timings and sizes of the last compress / factor / solve on this handle (HOST). */
int vbarms_get_stats(vbarms_t h, vbarms_fstats *st);

/* Device memory of the library in this process (HOST out[4]): bytes in use, bytes kept in
 * the library's cache for reuse, the peak of bytes in use, and the number of allocations
 * that reached the HIP runtime.  Freed buffers are cached per stream and reused for later
 * work on the same stream, so repeated factorizations of one matrix stop allocating after
 * the first.  Never fails. */
int vbarms_device_memory(int64_t *out);

/* enable != 0 (the default) replays the level launches of the last-level triangular
 * sweeps from a HIP graph captured at the first application after each factorization;
 * 0 launches them one by one.  Both give identical results.  Takes effect at the next
 * application. */
int vbarms_set_graphs(vbarms_t h, int32_t enable);

/* ---------------------------------------------------------------------------------- */
/* Kernel timing (measurement support).                                               */
/* ---------------------------------------------------------------------------------- */
/* Kernel classes timed with HIP events recorded on the handle's stream around their
 * launches, together with the algorithmic bytes each launch must move:
 *   VBARMS_K_SPMV   the FGMRES product A v (one VBSR SpMV launch)
 *   VBARMS_K_APPLY  one application of M^{-1} (all its launches)
 *   VBARMS_K_ILUT   one dependency wave of the last-level block ILUT
 *   VBARMS_K_TRSV   the two last-level block triangular sweeps of one application
 *   VBARMS_K_ORTHO  one classical Gram-Schmidt pass (dot products and update) */
#define VBARMS_K_SPMV 0
#define VBARMS_K_APPLY 1
#define VBARMS_K_ILUT 2
#define VBARMS_K_TRSV 3
#define VBARMS_K_ORTHO 4
#define VBARMS_K_COUNT 5

typedef struct {
    int64_t calls;   /* timed launches (or launch groups) */
    double ms;       /* summed event time, milliseconds */
    double bytes;    /* summed algorithmic bytes */
} vbarms_kstat;

/* enable != 0 starts recording (and clears the totals); 0 stops.  Recording adds two
 * event records per timed launch. */
int vbarms_set_timing(vbarms_t h, int32_t enable);
/* out[VBARMS_K_COUNT] (HOST): totals since timing was enabled; synchronizes the stream. */
int vbarms_kernel_stats(vbarms_t h, vbarms_kstat *out);

/* ---------------------------------------------------------------------------------- */
/* Inspection of the factors (for verification and analysis).  All outputs are HOST.  */
/* ---------------------------------------------------------------------------------- */
/* Matrices that can be exported (block sparse row, dense row-major blocks):
 *   VBARMS_M_A     A_l as handed to level l (A_0 = permuted input matrix)
 *   VBARMS_M_AS    S1 A_l S2 (scaled, level numbering)
 *   VBARMS_M_G     L^{-1} P F of level l (IS rows, remaining columns)
 *   VBARMS_M_W     E U^{-1} of level l (remaining rows, IS columns)
 *   VBARMS_M_D     LU factors of the IS pivot blocks of level l (block diagonal, pivots)
 *   VBARMS_M_LAST  matrix handed to the last-level ILUT
 *   VBARMS_M_L     last-level unit block lower factor (strictly lower blocks)
 *   VBARMS_M_U     last-level block upper factor without its diagonal blocks
 *   VBARMS_M_DL    LU factors of the last-level pivot blocks (block diagonal, pivots) */
#define VBARMS_M_A 0
#define VBARMS_M_AS 1
#define VBARMS_M_G 2
#define VBARMS_M_W 3
#define VBARMS_M_D 4
#define VBARMS_M_LAST 5
#define VBARMS_M_L 6
#define VBARMS_M_U 7
#define VBARMS_M_DL 8

/* levels actually factored */
int vbarms_num_levels(vbarms_t h, int32_t *levels);
/* info[5] = {p, n, nis, n_is, nis_sn} of level l: supernodes, rows, groups (pivot blocks
 * of D), rows of D, supernodes in the groups */
int vbarms_level_info(vbarms_t h, int32_t level, int32_t *info);
/* the independent-set supernodes of level l, group after group, members ascending, groups
 * by their smallest supernode (length nis_sn) */
int vbarms_level_is(vbarms_t h, int32_t level, int32_t *is_list);
/* gptr[nis+1]: group g is is_list[gptr[g] .. gptr[g+1]) */
int vbarms_level_groups(vbarms_t h, int32_t level, int32_t *gptr);
/* scaling vectors S1, S2 of level l (length n of the level) */
int vbarms_level_scaling(vbarms_t h, int32_t level, double *s1, double *s2);
/* dims[4] = {block rows, block columns, blocks, values} */
int vbarms_matrix_dims(vbarms_t h, int32_t which, int32_t level, int64_t *dims);
/* rb[p+1], cb[q+1]: scalar offsets of row/column blocks; rowptr[p+1], colidx[nb]: block
 * pattern with ascending columns; vals: blocks in order, each row-major; piv (D, DL only,
 * may be NULL): GEPP row interchanges, one per scalar row, local to the block. */
int vbarms_matrix_get(vbarms_t h, int32_t which, int32_t level, int32_t *rb, int32_t *cb,
                      int64_t *rowptr, int32_t *colidx, double *vals, int32_t *piv);

/* ---------------------------------------------------------------------------------- */
/* Learned parameter selection.  Not part of the paper's method: a small network that    */
/* predicts tau and the per-level drop tolerances from features of the matrix.  Callers */
/* that do not use it run the method with their own parameters.                          */
/* ---------------------------------------------------------------------------------- */
#define VBARMS_NFEAT 8

/* Features of A (DEVICE CSR as in vbarms_compress), f (HOST, VBARMS_NFEAT floats):
 *   0 log10 n                      4 smallest |a_ii| / sum_j |a_ij|
 *   1 mean row length / 100        5 share of entries below 1e-3 of their row's largest
 *   2 std / mean of row lengths    6 identical-pattern row classes per row
 *   3 mean |a_ii| / sum_j |a_ij|   7 mean |a_ij| (j != i) over |a_ii|
 * Leaves the handle's compressed matrix and factors untouched.  Errors: ARG (n = 0). */
int vbarms_features(vbarms_t h, const vbarms_csr *A, float *f);

/* Multilayer perceptron: in_dim -> `depth` dense ReLU layers of width `hidden` -> out_dim
 * (linear), FP32.  Parameters are packed layer by layer as W (n_out x n_in, row-major)
 * then b (n_out); they start at zero.  Training minimizes the mean squared error
 * sum (y - t)^2 / (batch * out_dim) with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * Work runs on `hip_stream`; every call returns after its work has finished. */
typedef struct vbarms_mlp_ctx *vbarms_mlp_t;
int vbarms_mlp_create(vbarms_mlp_t *m, int32_t in_dim, int32_t hidden, int32_t depth, int32_t out_dim,
                      void *hip_stream);
int vbarms_mlp_destroy(vbarms_mlp_t m);
const char *vbarms_mlp_last_error(vbarms_mlp_t m);
int vbarms_mlp_num_params(vbarms_mlp_t m, int64_t *n);
/* params: DEVICE, num_params floats.  set_params also clears the Adam moments. */
int vbarms_mlp_set_params(vbarms_mlp_t m, const float *params);
int vbarms_mlp_get_params(vbarms_mlp_t m, float *params);
/* x: DEVICE [batch x in_dim] row-major, y: DEVICE [batch x out_dim]. */
int vbarms_mlp_forward(vbarms_mlp_t m, const float *x, int32_t batch, float *y);
/* Loss (HOST, may be NULL) and gradient (DEVICE [num_params], may be NULL) for targets
 * t (DEVICE [batch x out_dim]); the gradient is kept for vbarms_mlp_adam_step. */
int vbarms_mlp_loss_grad(vbarms_mlp_t m, const float *x, const float *t, int32_t batch, float *loss,
                         float *grad);
/* One Adam update with the gradient of the last vbarms_mlp_loss_grad.  Errors: STATE if
 * there is none, ARG for lr <= 0. */
int vbarms_mlp_adam_step(vbarms_mlp_t m, float lr);

#ifdef __cplusplus
}
#endif
#endif /* VBARMS_H */
