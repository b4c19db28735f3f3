// y = A x (or y = b - A x) on the block-row panel layout.
//
// Each scalar row is a contiguous run of W_I values whose column list sc is shared by the
// m_I rows of its block row.  A group of TG lanes strides over one row (coalesced value
// reads, column indices served from cache for the sibling rows) and reduces with DPP
// shuffles.  HBM-bound: per call it moves the values, the shared column lists, x and y.
#include "common.h"

namespace vb {

namespace {

// NV vectors per launch row of the grid (blockIdx.y selects the group of NV vectors, each
// ld apart): every matrix value and column index is loaded once for the NV products.  The
// sum of every vector keeps the column order of the single-vector product.
template <class T, int TG, int NV>
__global__ void __launch_bounds__(256) k_spmv(int64_t n, const int *__restrict__ rowblk, const int *__restrict__ rb,
                                              const int64_t *__restrict__ wp, const int64_t *__restrict__ vp,
                                              const int *__restrict__ sc, const T *__restrict__ v,
                                              const double *__restrict__ x, const double *__restrict__ b,
                                              double *__restrict__ y, int nv, int64_t ld) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = gid / TG;
    int lane = (int)(gid % TG);
    const int v0 = blockIdx.y * NV;
    const int cnt = nv - v0 < NV ? nv - v0 : NV;
    const int64_t base = (int64_t)v0 * ld;
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = 0.0;
    if (row < n) {
        int I = rowblk[row];
        int rl = (int)(row - rb[I]);
        int64_t W = wp[I + 1] - wp[I];
        const T *a = v + vp[I] + rl * W;
        const int *c = sc + wp[I];
        const double *xv = x + base;
        for (int64_t j = lane; j < W; j += TG) {
            const double aj = (double)a[j];
            const int cj = c[j];
#pragma unroll
            for (int q = 0; q < NV; ++q)
                if (q < cnt) acc[q] += aj * xv[q * ld + cj];
        }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q)
#pragma unroll
        for (int off = TG / 2; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, TG);
    if (row < n && lane == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q)
            if (q < cnt) {
                const int64_t o = base + q * ld + row;
                y[o] = b ? b[o] - acc[q] : acc[q];
            }
}

template <class T, int TG>
void launch_spmv(const Panel<T> &a, int64_t n, const double *x, const double *b, double *y, int nv, int64_t ld,
                 hipStream_t s) {
    if (nv == 1) {
        k_spmv<T, TG, 1><<<grid_for(n * TG, 256), 256, 0, s>>>(n, a.rowblk.p, a.rb.p, a.wp.p, a.vp.p, a.sc.p, a.v.p,
                                                               x, b, y, 1, ld);
    } else {
        const dim3 grid(grid_for(n * TG, 256), (unsigned)((nv + 3) / 4));
        k_spmv<T, TG, 4><<<grid, 256, 0, s>>>(n, a.rowblk.p, a.rb.p, a.wp.p, a.vp.p, a.sc.p, a.v.p, x, b, y, nv, ld);
    }
    VB_LAUNCH_CHECK();
}

}  // namespace

// Lanes per scalar row: as many lanes as the autotuner picked for this matrix.  nv vectors
// (x, b and y each hold nv vectors of n entries, n apart) share the launch.
template <class T>
void panel_spmv_ex(const Panel<T> &a, const double *x, const double *b, double *y, hipStream_t s, int nv) {
    int64_t n = a.h_rb.empty() ? 0 : a.h_rb.back();
    if (n == 0 || nv < 1) return;
    switch (a.tg) {
    case 4: launch_spmv<T, 4>(a, n, x, b, y, nv, n, s); break;
    case 16: launch_spmv<T, 16>(a, n, x, b, y, nv, n, s); break;
    case 32: launch_spmv<T, 32>(a, n, x, b, y, nv, n, s); break;
    default: launch_spmv<T, 8>(a, n, x, b, y, nv, n, s); break;
    }
}

// Times the product with 4, 8, 16 and 32 lanes per scalar row on this matrix (one warm-up
// and five timed runs each, HIP events on the stream) and keeps the fastest.
template <class T>
int autotune_spmv(Panel<T> &a, hipStream_t s) {
    const int64_t n = a.h_rb.empty() ? 0 : a.h_rb.back();
    const int64_t ncol = a.h_cb.empty() ? 0 : a.h_cb.back();
    a.tg = 8;
    if (n == 0 || ncol == 0) return a.tg;
    DBuf<double> x(ncol), y(n);
    fill_val<double>(x.p, 1.0, ncol, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    VB_HIP(hipEventCreate(&e0));
    VB_HIP(hipEventCreate(&e1));
    float best = 0.f;
    int best_tg = 8;
    for (int tg : {4, 8, 16, 32}) {
        a.tg = tg;
        panel_spmv_ex<T>(a, x.p, nullptr, y.p, s, 1);
        VB_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 5; ++r) panel_spmv_ex<T>(a, x.p, nullptr, y.p, s, 1);
        VB_HIP(hipEventRecord(e1, s));
        VB_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        VB_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (tg == 4 || ms < best) {
            best = ms;
            best_tg = tg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    a.tg = best_tg;
    return best_tg;
}

// Bytes one product must move: the values, one column index per panel column, the
// per-block-row offsets (wp, vp, rb), x once, y (and b) once.
template <class T>
double panel_spmv_bytes(const Panel<T> &a, bool with_b) {
    double n = a.h_rb.empty() ? 0.0 : (double)a.h_rb.back();
    double ncol = a.h_cb.empty() ? 0.0 : (double)a.h_cb.back();
    return (double)sizeof(T) * (double)a.nv + 4.0 * (double)a.nw + 20.0 * (a.p + 1) + 8.0 * ncol +
           8.0 * n * (with_b ? 2.0 : 1.0);
}

template <class T>
void panel_spmv(const Panel<T> &a, const double *x, double *y, hipStream_t s, int nv) {
    panel_spmv_ex<T>(a, x, nullptr, y, s, nv);
}

template double panel_spmv_bytes<double>(const Panel<double> &, bool);
template double panel_spmv_bytes<float>(const Panel<float> &, bool);
template void panel_spmv<double>(const Panel<double> &, const double *, double *, hipStream_t, int);
template void panel_spmv<float>(const Panel<float> &, const double *, double *, hipStream_t, int);
template void panel_spmv_ex<double>(const Panel<double> &, const double *, const double *, double *, hipStream_t, int);
template void panel_spmv_ex<float>(const Panel<float> &, const double *, const double *, double *, hipStream_t, int);
template int autotune_spmv<double>(Panel<double> &, hipStream_t);
template int autotune_spmv<float>(Panel<float> &, hipStream_t);

}  // namespace vb
