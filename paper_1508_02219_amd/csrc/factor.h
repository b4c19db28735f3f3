// Multilevel factor data shared by the factorization, the solve and the C ABI.
#pragma once

#include "common.h"

namespace vb {

// One level of the partial block factorization (Sec. 3, Steps 2-4).
template <class T>
struct Level {
    int p = 0, n = 0;             // supernodes / scalar size of A_l
    int nis = 0, n_is = 0;        // pivot blocks of D (groups) / scalar size
    int nis_sn = 0;               // supernodes in the groups
    int nrest = 0, n_rest = 0;    // remaining supernodes / scalar size
    Panel<T> A;                   // A_l as received (kept for inspection)
    Panel<T> As;                  // S1 A_l S2
    DBuf<double> s1, s2;          // [n]
    DBuf<int> num;                // [p] position in the IS or in the rest
    DBuf<int> is_flag;            // [p]
    DBuf<int> is_list, rest_list; // ascending
    std::vector<int> h_is_rb, h_rest_rb;
    DBuf<int> is_rb, rest_rb;     // scalar offsets in the IS / rest numbering
    DBuf<int> is_rows, rest_rows; // [n_is], [n_rest]: level row of every IS / rest row
    std::vector<int> h_members;   // groups of several supernodes: members, group after group
    std::vector<int> h_gptr;      // [nis+1] into h_members (empty with one supernode per group)
    DBuf<T> dlu;                  // LU of the IS pivot blocks, concatenated
    DBuf<int64_t> dlu_off;        // [nis+1]
    DBuf<int> dpiv;               // [n_is] local row interchanges
    DBuf<int> dperm;              // [n_is] the interchanges as a permutation: row r of P x is x[dperm[r]]
    Panel<T> G;                   // L^{-1} P F: IS rows x rest columns
    Panel<T> W;                   // E U^{-1}:   rest rows x IS columns
    DBuf<double> y;               // apply workspace [n_is] per vector
    DBuf<double> t;               // apply workspace [n_is] per vector
    DBuf<double> g, z;            // apply workspace [n_rest] per vector: next level's right-hand side / solution
    int ws_nv = 0;                // vectors the apply workspaces hold
};

// An instantiated graph of captured launches (owned; destroyed with its owner).
struct LaunchGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    LaunchGraph() = default;
    LaunchGraph(const LaunchGraph &) = delete;
    LaunchGraph &operator=(const LaunchGraph &) = delete;
    ~LaunchGraph() { reset(); }
    void reset() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

// Last level block ILUT factors (Sec. 3, Alg. 3).
template <class T>
struct LastLevel {
    Panel<T> A;                   // matrix handed to the ILUT
    Panel<T> L, U;                // strictly lower multipliers / strictly upper blocks
    DBuf<T> dl;                   // LU of the pivot blocks
    DBuf<int64_t> dl_off;         // [p+1]
    DBuf<int> dl_piv;             // [n]
    std::vector<int> lorder, lptr;  // forward sweep: block rows sorted by level, level offsets
    std::vector<int> uorder, uptr;  // backward sweep
    DBuf<int64_t> d_lrows, d_urows; // row descriptors of the two sweeps, in sweep order
    int waves = 0;                  // kernel launches the factorization took
    int attempts = 0;               // runs of the factorization (more than one after a capacity retry)
    double sweep_bytes = 0;         // algorithmic bytes of one forward + backward sweep
    DBuf<double> t;               // solve workspace [n]
    // the two sweeps captured once as a graph that reads gb and writes gx
    bool use_graph = true;
    LaunchGraph sweeps;
    DBuf<double> gb, gx;          // [n]
    // the same for several vectors at once (mv_nv vectors, n apart)
    int mv_nv = 0;
    LaunchGraph sweeps_mv;
    DBuf<double> t_mv, gb_mv, gx_mv;
};

template <class T>
struct Factors {
    std::vector<Level<T>> lev;
    LastLevel<T> last;
    int nlev = 0;
    double level_ms[VBARMS_MAX_LEVELS] = {0};
    double ilut_ms = 0;
    double apply_bytes = 0;       // algorithmic bytes of one application of M^{-1}
};

// device error record: {code, level, block, aux}
struct DevErr {
    DBuf<int> rec;
    void reset(hipStream_t s) {
        if (!rec.p) rec.alloc(4);
        VB_HIP(hipMemsetAsync(rec.p, 0, 4 * sizeof(int), s));
    }
};

// Lexicographically first maximal independent set of a graph given by one or two
// adjacency lists (state: 1 in the set, 2 out).  The visiting order is ascending vertex
// number, or, when prio is given, descending prio with ties in ascending number.
void lfmis(int nv, const int64_t *eptr, const int *elist, const int64_t *eptr2, const int *elist2, const double *prio,
           int *state, hipStream_t s);
std::vector<int> compress_gpu(int n, const int64_t *rowptr, const int *col, double tau, int *perm, hipStream_t s);
// Graph-based compression with target average block density mu on a host copy of the
// pattern; returns the block offsets and fills perm (new position -> original row).
std::vector<int> graph_compress_host(int n, const std::vector<int64_t> &rp, const std::vector<int> &ci, double mu,
                                     std::vector<int> &perm);
void panel_from_csr(int n, const int64_t *rowptr, const int *col, const double *val, const int *perm,
                    const std::vector<int> &bptr, Panel<double> &out, int *err, hipStream_t s);
template <class T>
void panel_spmv_ex(const Panel<T> &a, const double *x, const double *b, double *y, hipStream_t s, int nv = 1);
template <class Tin, class Tout>
void panel_convert(const Panel<Tin> &src, Panel<Tout> &dst, hipStream_t s);

// Factors level `lvl` of A (consumed), producing the next Schur complement in `next`.
// Pivot blocks whose pivot ratio (smallest over largest pivot magnitude) falls below
// min_ratio are counted in err[3].
template <class T>
void factor_level(Level<T> &L, Panel<T> &&A, int lvl, double droptol, int drop_schur, int is_order, int group_rows,
                  double min_ratio, Panel<T> &next, int *err, hipStream_t s);
// Room reserved by the block ILUT, kept by the caller across factorizations: working rows
// hold `grow` times their input row (and at least `grow` times the mean row); the L and U
// pools hold `pool` times the input's blocks and values each; a row's block list in LDS
// holds `rbcap` entries.  All only grow, when an attempt runs out of room.
struct IlutHint {
    int grow = 4;
    double pool = 1.5;
    int rbcap = 256;  // block-list entries a row may hold in LDS
};
// Block ILUT of `last.A` with threshold t.
template <class T>
void factor_last(LastLevel<T> &last, double droptol, double min_ratio, int lvl, IlutHint &hint, int *err,
                 hipStream_t s);
// x = U^{-1} L^{-1} b for the last level (b and x may alias)
template <class T>
void solve_last(LastLevel<T> &last, const double *b, double *x, int *err, hipStream_t s, int nv = 1);
// x_l = M_l^{-1} b_l recursively from level `lvl` (vectors in the level's numbering)
template <class T>
void solve_levels(Factors<T> &f, int lvl, const double *b, double *x, int nv, int *err, hipStream_t s);

}  // namespace vb

#include <functional>

namespace vb {

struct KrylovWork {
    DBuf<double> V, Z, partial, hdev, nrm;
    int64_t n = 0;
    int m = 0;
    void ensure(int64_t n_, int m_);
};
int fgmres_run(const Panel<double> &A, KrylovWork &kw, const double *b, double *x, double tol, int m, int maxit,
               const std::function<void(const double *, double *)> &precond, vbarms_sinfo *info, hipStream_t s);

// Consecutive row ranges of independent systems inside one combined numbering, with the
// chunking used by the per-system dot products (batch.hip).
struct Segments {
    int nseg = 0, nchunk = 0;
    std::vector<int64_t> off;          // [nseg+1]
    DBuf<int64_t> d_off, d_cbeg, d_cend;
    DBuf<int> d_segchunk;              // [nseg+1] first chunk of every segment
    DBuf<int> rowseg;                  // [n] segment of every row
    void build(const std::vector<int64_t> &offsets, hipStream_t s);
};
struct BatchKrylovWork {
    DBuf<double> V, Z, partial, hbuf, ybuf;
    DBuf<int> ibuf;
    int64_t n = 0;
    int m = 0, nseg = 0, nchunk = 0;
    void ensure(int64_t n_, int m_, int nseg_, int nchunk_);
};
// FGMRES(m) on every segment of A (block diagonal over the segments) in lockstep; info[s]
// per system.  Returns VBARMS_OK when every system converged.
// Lockstep FGMRES over nv copies of the combined system at once: b and x hold nv vectors of
// A's size one after another, sg segments that long numbering (every system of every
// vector), and precond(in, out, nv) applies M^{-1} to nv vectors.
int fgmres_batch_run(const Panel<double> &A, int nv, BatchKrylovWork &kw, const Segments &sg, const double *b,
                     double *x, double tol, int m, int maxit,
                     const std::function<void(const double *, double *, int)> &precond,
                     std::vector<vbarms_sinfo> &info, hipStream_t s);
void gather_perm(int n, const int *perm, const double *src, double *dst, hipStream_t s);
// VBARMS_NFEAT features of a CSR matrix (host output)
void matrix_features(int n, int64_t nnz, const int64_t *rowptr, const int *col, const double *val, float *f,
                     hipStream_t s);
void scatter_perm(int n, const int *perm, const double *src, double *dst, hipStream_t s);

}  // namespace vb
