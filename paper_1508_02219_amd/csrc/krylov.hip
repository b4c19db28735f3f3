// Right-preconditioned FGMRES(m) (Sec. 4.1) in FP64 with classical Gram-Schmidt applied
// twice.  The Krylov vectors V (m+1 x n) and the preconditioned vectors Z (m x n) stay in
// HBM; one short device-to-host copy per Arnoldi step brings the new Hessenberg column to
// the host, where the Givens rotations run.  All dot products are reduced in a fixed
// order (per-block partials, then a per-column sum), so results are deterministic.
#include <cmath>

#include "factor.h"

namespace vb {

namespace {

constexpr int kDotThreads = 256;
constexpr int kDotBlocks = 512;

// partial[b * ncols + k] = sum over block b's elements of V_k . w
__global__ void __launch_bounds__(kDotThreads) k_dots(int64_t n, int ncols, const double *V, int64_t ldv,
                                                      const double *w, double *partial) {
    __shared__ double red[kDotThreads / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    for (int k = 0; k < ncols; ++k) {
        const double *v = V + (int64_t)k * ldv;
        double s = 0.0;
        for (int64_t i = (int64_t)blockIdx.x * kDotThreads + t; i < n; i += (int64_t)gridDim.x * kDotThreads)
            s += v[i] * w[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int q = 0; q < kDotThreads / 64; ++q) tot += red[q];
            partial[(int64_t)blockIdx.x * ncols + k] = tot;
        }
        __syncthreads();
    }
}
// out[k] (+)= sum_b partial[b * ncols + k]
__global__ void k_dot_reduce(int nblk, int ncols, const double *partial, double *out, int accumulate) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ncols) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * ncols + k];
    out[k] = accumulate ? out[k] + s : s;
}
// w -= sum_k h[k] V_k
__global__ void k_update(int64_t n, int ncols, const double *V, int64_t ldv, const double *h, double *w) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int k = 0; k < ncols; ++k) s -= h[k] * V[(int64_t)k * ldv + i];
    w[i] = s;
}
__global__ void k_scale_copy(int64_t n, const double *w, const double *den, double *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = *den;
    out[i] = d > 0.0 ? w[i] / d : w[i];
}
__global__ void k_sqrt_inplace(double *x) { *x = sqrt(*x); }
__global__ void k_xupdate(int64_t n, int ncols, const double *Z, int64_t ldz, const double *y, double *x) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = x[i];
    for (int k = 0; k < ncols; ++k) s += y[k] * Z[(int64_t)k * ldz + i];
    x[i] = s;
}
__global__ void k_gather(int n, const int *perm, const double *src, double *dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}
__global__ void k_scatter(int n, const int *perm, const double *src, double *dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

}  // namespace

void gather_perm(int n, const int *perm, const double *src, double *dst, hipStream_t s) {
    if (n <= 0) return;
    k_gather<<<grid_for(n, 256), 256, 0, s>>>(n, perm, src, dst);
    VB_LAUNCH_CHECK();
}
void scatter_perm(int n, const int *perm, const double *src, double *dst, hipStream_t s) {
    if (n <= 0) return;
    k_scatter<<<grid_for(n, 256), 256, 0, s>>>(n, perm, src, dst);
    VB_LAUNCH_CHECK();
}

void KrylovWork::ensure(int64_t n_, int m_) {
    if (n_ == n && m_ == m) return;
    n = n_;
    m = m_;
    V.alloc((size_t)(m + 1) * std::max<int64_t>(n, 1));
    Z.alloc((size_t)m * std::max<int64_t>(n, 1));
    partial.alloc((size_t)kDotBlocks * (m + 2));
    hdev.alloc(2 * (m + 2));
    nrm.alloc(2);
}

// dots of w with the first ncols columns of V into out (device)
static void multidot(KrylovWork &kw, int64_t n, int ncols, const double *V, const double *w, double *out,
                     int accumulate, hipStream_t s) {
    k_dots<<<kDotBlocks, kDotThreads, 0, s>>>(n, ncols, V, n, w, kw.partial.p);
    VB_LAUNCH_CHECK();
    k_dot_reduce<<<grid_for(ncols, 64), 64, 0, s>>>(kDotBlocks, ncols, kw.partial.p, out, accumulate);
    VB_LAUNCH_CHECK();
}

// Solves A x = b in the compressed numbering.  `precond` applies M^{-1} (in, out).
int fgmres_run(const Panel<double> &A, KrylovWork &kw, const double *b, double *x, double tol, int m, int maxit,
               const std::function<void(const double *, double *)> &precond, vbarms_sinfo *info, hipStream_t s) {
    const int64_t n = A.h_rb.empty() ? 0 : A.h_rb.back();
    kw.ensure(n, m);
    double *V = kw.V.p, *Z = kw.Z.p;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), yv(m + 1), hcol(2 * (m + 2));
    multidot(kw, n, 1, b, b, kw.nrm.p, 0, s);
    k_sqrt_inplace<<<1, 1, 0, s>>>(kw.nrm.p);
    double bn = read_one(kw.nrm.p, s);
    if (!std::isfinite(bn)) fail(VBARMS_ERR_NAN, "right-hand side contains NaN or Inf");
    int it = 0, restarts = 0, status = VBARMS_NOT_CONVERGED;
    double rel = 0.0;
    if (bn == 0.0) {
        if (n) VB_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
        status = VBARMS_OK;
    } else {
        for (;;) {
            {
                KScope ks(VBARMS_K_SPMV, panel_spmv_bytes(A, true), s);
                panel_spmv_ex<double>(A, x, b, V, s);  // V0 = b - A x
            }
            multidot(kw, n, 1, V, V, kw.nrm.p, 0, s);
            k_sqrt_inplace<<<1, 1, 0, s>>>(kw.nrm.p);
            double beta = read_one(kw.nrm.p, s);
            if (!std::isfinite(beta)) fail(VBARMS_ERR_NAN, "residual became NaN or Inf");
            rel = beta / bn;
            if (rel <= tol) { status = VBARMS_OK; break; }
            if (it >= maxit) break;
            k_scale_copy<<<grid_for(n, 256), 256, 0, s>>>(n, V, kw.nrm.p, V);
            VB_LAUNCH_CHECK();
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int j = 0;
            for (; j < m && it < maxit; ++j) {
                double *vj = V + (int64_t)j * n, *zj = Z + (int64_t)j * n, *vn = V + (int64_t)(j + 1) * n;
                precond(vj, zj);
                {
                    KScope ks(VBARMS_K_SPMV, panel_spmv_bytes(A, false), s);
                    panel_spmv<double>(A, zj, vn, s);
                }
                double *h1 = kw.hdev.p, *h2 = kw.hdev.p + (m + 2);
                // one pass reads V_0..V_j twice (dots, update) and w three times
                const double pass_bytes = 8.0 * (double)n * (2.0 * (j + 1) + 3.0);
                {
                    KScope ks(VBARMS_K_ORTHO, pass_bytes, s);
                    multidot(kw, n, j + 1, V, vn, h1, 0, s);
                    k_update<<<grid_for(n, 256), 256, 0, s>>>(n, j + 1, V, n, h1, vn);
                    VB_LAUNCH_CHECK();
                }
                {
                    KScope ks(VBARMS_K_ORTHO, pass_bytes, s);
                    multidot(kw, n, j + 1, V, vn, h2, 0, s);
                    k_update<<<grid_for(n, 256), 256, 0, s>>>(n, j + 1, V, n, h2, vn);
                    VB_LAUNCH_CHECK();
                }
                multidot(kw, n, 1, vn, vn, kw.nrm.p, 0, s);
                k_sqrt_inplace<<<1, 1, 0, s>>>(kw.nrm.p);
                k_scale_copy<<<grid_for(n, 256), 256, 0, s>>>(n, vn, kw.nrm.p, vn);
                VB_LAUNCH_CHECK();
                VB_HIP(hipMemcpyAsync(hcol.data(), kw.hdev.p, sizeof(double) * 2 * (m + 2), hipMemcpyDeviceToHost, s));
                double hn = 0.0;
                VB_HIP(hipMemcpyAsync(&hn, kw.nrm.p, sizeof(double), hipMemcpyDeviceToHost, s));
                VB_HIP(hipStreamSynchronize(s));
                for (int k = 0; k <= j; ++k) H[k * m + j] = hcol[k] + hcol[(m + 2) + k];
                H[(j + 1) * m + j] = hn;
                for (int k = 0; k < j; ++k) {
                    double a = H[k * m + j], c = H[(k + 1) * m + j];
                    H[k * m + j] = cs[k] * a + sn[k] * c;
                    H[(k + 1) * m + j] = -sn[k] * a + cs[k] * c;
                }
                double a = H[j * m + j], c = H[(j + 1) * m + j];
                double r = std::sqrt(a * a + c * c);
                cs[j] = r > 0.0 ? a / r : 1.0;
                sn[j] = r > 0.0 ? c / r : 0.0;
                H[j * m + j] = r;
                H[(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++it;
                if (!std::isfinite(g[j + 1])) fail(VBARMS_ERR_NAN, "Arnoldi produced NaN or Inf");
                if (std::fabs(g[j + 1]) <= tol * bn || hn == 0.0) { ++j; break; }
            }
            for (int k = j - 1; k >= 0; --k) {
                double sum = g[k];
                for (int q = k + 1; q < j; ++q) sum -= H[k * m + q] * yv[q];
                yv[k] = sum / H[k * m + k];
            }
            VB_HIP(hipMemcpyAsync(kw.hdev.p, yv.data(), sizeof(double) * j, hipMemcpyHostToDevice, s));
            k_xupdate<<<grid_for(n, 256), 256, 0, s>>>(n, j, Z, n, kw.hdev.p, x);
            VB_LAUNCH_CHECK();
            ++restarts;
        }
    }
    if (info) {
        info->iters = it;
        info->restarts = restarts;
        info->true_relres = rel;
        info->status = status;
        info->fp64_refactor = 0;
    }
    return status;
}

}  // namespace vb
