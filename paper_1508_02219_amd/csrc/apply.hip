// The multilevel solve (Alg. 2) with the scalings and permutations of every level.
//
// At level l, with b_l in the level's numbering (is_rows / rest_rows give the level row of
// every row of the IS and rest numberings; a pivot block is one group of supernodes):
//   f = (S1 b)_IS,  y_i = L_i^{-1} P_i f_i              one lane per pivot block
//   g' = (S1 b)_rest - W y                             row-streamed SpMV with W
//   z = next level (or the last-level block ILUT solve) on g'
//   u_i = U_i^{-1} (y - G z)_i                         row-streamed SpMV with G, then per block
//   x_l = S2 P_I^T (u, z)
// Several vectors go through at once: every kernel takes the vector from blockIdx.y, each
// array holding its vectors one after another (ld apart).
#include "factor.h"

namespace vb {

namespace {

constexpr int kTG = 8;

template <class T>
__global__ void __launch_bounds__(64) k_lvl_down(int nis, const int *is_rows, const int *is_rb, const double *s1,
                                                 const double *b, int64_t ldb, const T *dlu, const int64_t *dlu_off,
                                                 const int *dperm, double *y, int64_t ldy) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nis) return;
    b += blockIdx.y * ldb;
    y += blockIdx.y * ldy;
    const int m = is_rb[i + 1] - is_rb[i];
    const int *rows = is_rows + is_rb[i];
    const int *pm = dperm + is_rb[i];
    double x[VBARMS_MAX_BLOCK];  // P (S1 b) of the block, the exchanges applied while loading
#pragma unroll
    for (int r = 0; r < VBARMS_MAX_BLOCK; ++r) {
        if (r < m) {
            const int row = rows[pm[r]];
            x[r] = s1[row] * b[row];
        } else {
            x[r] = 0.0;
        }
    }
    reg_l_fwd<T, double, VBARMS_MAX_BLOCK>(m, dlu + dlu_off[i], x);
#pragma unroll
    for (int r = 0; r < VBARMS_MAX_BLOCK; ++r)
        if (r < m) y[is_rb[i] + r] = x[r];
}

// out[rr] = s1[row(rr)] base[row(rr)] - sum_c P[rr, c] v[sc[c]], with row(rr) = rows[rr]
// the level row of panel row rr (rows == nullptr: out[rr] = base[rr] - ...)
template <class T>
__global__ void __launch_bounds__(256) k_lvl_spmv(int64_t nrows, const int *rowblk, const int *prb, const int64_t *wp,
                                                  const int64_t *vp, const int *sc, const T *pv, const double *v,
                                                  int64_t ldv, const int *rows, const double *s1, const double *base,
                                                  int64_t ldbase, double *out, int64_t ldout) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    v += blockIdx.y * ldv;
    base += blockIdx.y * ldbase;
    out += blockIdx.y * ldout;
    int64_t rr = gid / kTG;
    int lane = (int)(gid % kTG);
    double acc = 0.0;
    int I = 0;
    if (rr < nrows) {
        I = rowblk[rr];
        int64_t W = wp[I + 1] - wp[I];
        const T *a = pv + vp[I] + (rr - prb[I]) * W;
        const int *c = sc + wp[I];
        for (int64_t j = lane; j < W; j += kTG) acc += (double)a[j] * v[c[j]];
    }
#pragma unroll
    for (int off = kTG / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kTG);
    if (rr < nrows && lane == 0) {
        double bv;
        if (rows) {
            const int row = rows[rr];
            bv = s1[row] * base[row];
        } else {
            bv = base[rr];
        }
        out[rr] = bv - acc;
    }
}

template <class T>
__global__ void __launch_bounds__(64) k_lvl_up(int nis, const int *is_rows, const int *is_rb, const double *s2,
                                               const T *dlu, const int64_t *dlu_off, const double *t, int64_t ldt,
                                               double *x, int64_t ldx) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nis) return;
    t += blockIdx.y * ldt;
    x += blockIdx.y * ldx;
    const int m = is_rb[i + 1] - is_rb[i];
    const int *rows = is_rows + is_rb[i];
    double u[VBARMS_MAX_BLOCK];
#pragma unroll
    for (int r = 0; r < VBARMS_MAX_BLOCK; ++r) u[r] = r < m ? t[is_rb[i] + r] : 0.0;
    reg_lu_bwd<T, double, VBARMS_MAX_BLOCK>(m, dlu + dlu_off[i], u);
#pragma unroll
    for (int r = 0; r < VBARMS_MAX_BLOCK; ++r)
        if (r < m) x[rows[r]] = s2[rows[r]] * u[r];
}

__global__ void k_lvl_rest_out(int64_t nrest_rows, const int *rest_rows, const double *s2, const double *z,
                               int64_t ldz, double *x, int64_t ldx) {
    int64_t rr = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (rr >= nrest_rows) return;
    z += blockIdx.y * ldz;
    x += blockIdx.y * ldx;
    const int row = rest_rows[rr];
    x[row] = s2[row] * z[rr];
}

}  // namespace

template <class T>
void solve_levels(Factors<T> &f, int lvl, const double *b, double *x, int nv, int *err, hipStream_t s) {
    if (lvl == f.nlev) {
        solve_last(f.last, b, x, err, s, nv);
        return;
    }
    Level<T> &L = f.lev[lvl];
    if (L.ws_nv < nv) {  // workspaces for nv vectors
        L.y.alloc((size_t)std::max(L.n_is, 1) * nv);
        L.t.alloc((size_t)std::max(L.n_is, 1) * nv);
        L.g.alloc((size_t)std::max(L.n_rest, 1) * nv);
        L.z.alloc((size_t)std::max(L.n_rest, 1) * nv);
        L.ws_nv = nv;
    }
    const int64_t n = L.n, nis = L.n_is, nr = L.n_rest;
    const unsigned vy = (unsigned)nv;
    if (L.nis > 0) {
        k_lvl_down<T><<<dim3(grid_for(L.nis, 64), vy), 64, 0, s>>>(L.nis, L.is_rows.p, L.is_rb.p, L.s1.p, b, n,
                                                                    L.dlu.p, L.dlu_off.p, L.dperm.p, L.y.p, nis);
        VB_LAUNCH_CHECK();
    }
    if (L.n_rest > 0) {
        k_lvl_spmv<T><<<dim3(grid_for((int64_t)L.n_rest * kTG, 256), vy), 256, 0, s>>>(
            L.n_rest, L.W.rowblk.p, L.W.rb.p, L.W.wp.p, L.W.vp.p, L.W.sc.p, L.W.v.p, L.y.p, nis, L.rest_rows.p, L.s1.p,
            b, n, L.g.p, nr);
        VB_LAUNCH_CHECK();
    }
    solve_levels(f, lvl + 1, L.g.p, L.z.p, nv, err, s);
    if (L.nis > 0) {
        k_lvl_spmv<T><<<dim3(grid_for((int64_t)L.n_is * kTG, 256), vy), 256, 0, s>>>(
            L.n_is, L.G.rowblk.p, L.G.rb.p, L.G.wp.p, L.G.vp.p, L.G.sc.p, L.G.v.p, L.z.p, nr, nullptr, nullptr, L.y.p,
            nis, L.t.p, nis);
        VB_LAUNCH_CHECK();
        k_lvl_up<T><<<dim3(grid_for(L.nis, 64), vy), 64, 0, s>>>(L.nis, L.is_rows.p, L.is_rb.p, L.s2.p, L.dlu.p,
                                                                  L.dlu_off.p, L.t.p, nis, x, n);
        VB_LAUNCH_CHECK();
    }
    if (L.n_rest > 0) {
        k_lvl_rest_out<<<dim3(grid_for(L.n_rest, 256), vy), 256, 0, s>>>(L.n_rest, L.rest_rows.p, L.s2.p, L.z.p, nr,
                                                                          x, n);
        VB_LAUNCH_CHECK();
    }
}

template void solve_levels<double>(Factors<double> &, int, const double *, double *, int, int *, hipStream_t);
template void solve_levels<float>(Factors<float> &, int, const double *, double *, int, int *, hipStream_t);

}  // namespace vb
