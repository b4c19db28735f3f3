// Batched solves of independent systems (several systems factored as one block-diagonal
// matrix) with right-preconditioned FGMRES(m) run for all of them, and for several
// right-hand sides, in lockstep: every kernel of a step covers every system and vector,
// while the inner products, the Hessenberg matrices, the Givens rotations, convergence and
// restarts are kept per system and vector.
//
// Systems occupy consecutive row ranges ("segments") of the combined numbering.  The dot
// products are reduced per segment in a fixed order (chunk partials, then the chunks of a
// segment in order), so results are deterministic.
#include <algorithm>
#include <cmath>

#include "factor.h"

namespace vb {

namespace {

constexpr int kSegThreads = 256;
constexpr int kChunk = 16384;  // rows of one chunk of a segment

// partial[c * ncols + k] = sum over the rows of chunk c of V_k . w
__global__ void __launch_bounds__(kSegThreads) k_seg_dots(int nchunk, const int64_t *cbeg, const int64_t *cend,
                                                          int ncols, const double *V, int64_t ldv, const double *w,
                                                          double *partial) {
    __shared__ double red[kSegThreads / 64];
    const int c = blockIdx.x;
    if (c >= nchunk) return;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t b = cbeg[c], e = cend[c];
    for (int k = 0; k < ncols; ++k) {
        const double *v = V + (int64_t)k * ldv;
        double s = 0.0;
        for (int64_t i = b + t; i < e; i += kSegThreads) s += v[i] * w[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int q = 0; q < kSegThreads / 64; ++q) tot += red[q];
            partial[(int64_t)c * ncols + k] = tot;
        }
        __syncthreads();
    }
}
// out[s * ld + k] = sum of the partials of segment s's chunks (in chunk order)
__global__ void k_seg_reduce(int nseg, int ncols, const int *seg_chunk, const double *partial, double *out, int ld) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nseg * ncols) return;
    const int sg = q / ncols, k = q - sg * ncols;
    double s = 0.0;
    for (int c = seg_chunk[sg]; c < seg_chunk[sg + 1]; ++c) s += partial[(int64_t)c * ncols + k];
    out[(int64_t)sg * ld + k] = s;
}
// w_i -= sum_k h[s(i) * ld + k] V_k[i]
__global__ void k_seg_update(int64_t n, const int *rowseg, int ncols, const double *V, int64_t ldv, const double *h,
                             int ld, double *w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *hs = h + (int64_t)rowseg[i] * ld;
    double s = w[i];
    for (int k = 0; k < ncols; ++k) s -= hs[k] * V[(int64_t)k * ldv + i];
    w[i] = s;
}
// out_i = w_i / den[s(i)] (0 where the segment's norm is 0 or the segment is inactive)
__global__ void k_seg_scale(int64_t n, const int *rowseg, const double *w, const double *den, int ld,
                            const int *active, double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sg = rowseg[i];
    const double d = den[(int64_t)sg * ld];
    out[i] = active[sg] && d > 0.0 ? w[i] / d : 0.0;
}
// x_i += sum_{k < nk[s(i)]} y[s(i) * ld + k] Z_k[i]
__global__ void k_seg_xupdate(int64_t n, const int *rowseg, const int *nk, const double *Z, int64_t ldz,
                              const double *y, int ld, double *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sg = rowseg[i];
    const double *ys = y + (int64_t)sg * ld;
    double s = x[i];
    for (int k = 0; k < nk[sg]; ++k) s += ys[k] * Z[(int64_t)k * ldz + i];
    x[i] = s;
}
__global__ void k_rowseg(int nseg, const int64_t *off, int *rowseg) {
    const int sg = blockIdx.x;
    if (sg >= nseg) return;
    for (int64_t i = off[sg] + threadIdx.x; i < off[sg + 1]; i += blockDim.x) rowseg[i] = sg;
}

}  // namespace

void Segments::build(const std::vector<int64_t> &offsets, hipStream_t s) {
    off = offsets;
    nseg = (int)off.size() - 1;
    const int64_t n = off.back();
    std::vector<int64_t> cb, ce;
    std::vector<int> sc(nseg + 1, 0);
    for (int g = 0; g < nseg; ++g) {
        sc[g] = (int)cb.size();
        for (int64_t b = off[g]; b < off[g + 1]; b += kChunk) {
            cb.push_back(b);
            ce.push_back(std::min<int64_t>(off[g + 1], b + kChunk));
        }
    }
    sc[nseg] = (int)cb.size();
    nchunk = (int)cb.size();
    d_off.alloc(nseg + 1);
    to_device(d_off.p, off.data(), nseg + 1, s);
    d_cbeg.alloc(std::max(nchunk, 1));
    d_cend.alloc(std::max(nchunk, 1));
    d_segchunk.alloc(nseg + 1);
    if (nchunk) {
        to_device(d_cbeg.p, cb.data(), nchunk, s);
        to_device(d_cend.p, ce.data(), nchunk, s);
    }
    to_device(d_segchunk.p, sc.data(), nseg + 1, s);
    rowseg.alloc(std::max<int64_t>(n, 1));
    if (nseg > 0) {
        k_rowseg<<<nseg, 256, 0, s>>>(nseg, d_off.p, rowseg.p);
        VB_LAUNCH_CHECK();
    }
    VB_HIP(hipStreamSynchronize(s));  // host vectors above are copy sources
}

// out[s * ld + k] = <V_k, w>_s for k < ncols (device), through the chunk partials
static void seg_dots(const Segments &sg, BatchKrylovWork &kw, int64_t ldv, int ncols, const double *V, const double *w,
                     double *out, int ld, hipStream_t s) {
    if (sg.nchunk == 0) return;
    k_seg_dots<<<sg.nchunk, kSegThreads, 0, s>>>(sg.nchunk, sg.d_cbeg.p, sg.d_cend.p, ncols, V, ldv, w, kw.partial.p);
    VB_LAUNCH_CHECK();
    k_seg_reduce<<<grid_for((int64_t)sg.nseg * ncols, 256), 256, 0, s>>>(sg.nseg, ncols, sg.d_segchunk.p, kw.partial.p,
                                                                         out, ld);
    VB_LAUNCH_CHECK();
}

void BatchKrylovWork::ensure(int64_t n_, int m_, int nseg_, int nchunk_) {
    if (n_ != n || m_ != m) {
        n = n_;
        m = m_;
        V.alloc((size_t)(m + 1) * std::max<int64_t>(n, 1));
        Z.alloc((size_t)m * std::max<int64_t>(n, 1));
    }
    if (nseg_ != nseg || nchunk_ != nchunk || (int)hbuf.n < 3 * nseg_ * (m + 2)) {
        nseg = nseg_;
        nchunk = nchunk_;
        partial.alloc((size_t)std::max(nchunk, 1) * (m + 2));
        hbuf.alloc((size_t)3 * std::max(nseg, 1) * (m + 2));
        ybuf.alloc((size_t)std::max(nseg, 1) * (m + 1));
        ibuf.alloc((size_t)2 * std::max(nseg, 1));
    }
}

int fgmres_batch_run(const Panel<double> &A, int nv, BatchKrylovWork &kw, const Segments &sg, const double *b,
                     double *x, double tol, int m, int maxit,
                     const std::function<void(const double *, double *, int)> &precond,
                     std::vector<vbarms_sinfo> &info, hipStream_t s) {
    const int64_t n = (A.h_rb.empty() ? 0 : A.h_rb.back()) * (int64_t)nv;
    const int ns = sg.nseg;
    kw.ensure(n, m, ns, sg.nchunk);
    double *V = kw.V.p, *Z = kw.Z.p;
    const int ld = m + 2;  // stride of the per-segment coefficient rows
    double *h1 = kw.hbuf.p, *h2 = kw.hbuf.p + (size_t)ns * ld, *hn = kw.hbuf.p + 2 * (size_t)ns * ld;
    int *d_active = kw.ibuf.p, *d_nk = kw.ibuf.p + ns;
    info.assign(ns, vbarms_sinfo{});
    std::vector<double> bn(ns), beta(ns);
    std::vector<std::vector<double>> H(ns), cs(ns), sn(ns), g(ns);
    std::vector<int> active(ns, 1), running(ns, 0), nk(ns, 0), hact(ns);
    std::vector<double> hcopy((size_t)3 * ns * ld), yall((size_t)ns * (m + 1), 0.0);
    auto norms = [&](const double *w, std::vector<double> &out) {
        seg_dots(sg, kw, n, 1, w, w, hn, ld, s);
        std::vector<double> tmp((size_t)ns * ld);
        if (ns) VB_HIP(hipMemcpyAsync(tmp.data(), hn, sizeof(double) * ns * ld, hipMemcpyDeviceToHost, s));
        VB_HIP(hipStreamSynchronize(s));
        for (int q = 0; q < ns; ++q) out[q] = std::sqrt(tmp[(size_t)q * ld]);
    };
    auto upload_active = [&](const std::vector<int> &flags) {
        to_device(d_active, flags.data(), ns, s);
    };
    norms(b, bn);
    for (int q = 0; q < ns; ++q) {
        if (!std::isfinite(bn[q])) fail(VBARMS_ERR_NAN, "right-hand side contains NaN or Inf");
        if (bn[q] == 0.0) {
            active[q] = 0;
            info[q].status = VBARMS_OK;
        } else {
            info[q].status = VBARMS_NOT_CONVERGED;
        }
        H[q].assign((size_t)(m + 1) * m, 0.0);
        cs[q].assign(m, 0.0);
        sn[q].assign(m, 0.0);
        g[q].assign(m + 1, 0.0);
    }
    {
        // x = 0 for the systems with b = 0 (they are solved): x is scaled by 1 where b != 0
        // and set to 0 elsewhere
        std::vector<int> nonzero(ns);
        std::vector<double> one((size_t)ns * ld, 1.0);
        for (int q = 0; q < ns; ++q) nonzero[q] = bn[q] != 0.0;
        upload_active(nonzero);
        to_device(hn, one.data(), (size_t)ns * ld, s);
        k_seg_scale<<<grid_for(n, 256), 256, 0, s>>>(n, sg.rowseg.p, x, hn, ld, d_active, x);
        VB_LAUNCH_CHECK();
        VB_HIP(hipStreamSynchronize(s));  // the host vectors are the copy sources
    }
    int it = 0;
    for (;;) {
        // residuals of every system; converged ones stop
        panel_spmv_ex<double>(A, x, b, V, s, nv);  // V0 = b - A x
        norms(V, beta);
        bool any = false;
        for (int q = 0; q < ns; ++q) {
            if (!active[q]) continue;
            if (!std::isfinite(beta[q])) fail(VBARMS_ERR_NAN, "residual became NaN or Inf");
            info[q].true_relres = beta[q] / bn[q];
            if (info[q].true_relres <= tol) {
                active[q] = 0;
                info[q].status = VBARMS_OK;
            } else {
                any = true;
            }
        }
        if (!any || it >= maxit) break;
        // V0 /= beta per active system
        {
            std::vector<double> den((size_t)ns * ld, 0.0);
            for (int q = 0; q < ns; ++q) den[(size_t)q * ld] = beta[q];
            to_device(hn, den.data(), (size_t)ns * ld, s);
            upload_active(active);
            k_seg_scale<<<grid_for(n, 256), 256, 0, s>>>(n, sg.rowseg.p, V, hn, ld, d_active, V);
            VB_LAUNCH_CHECK();
            VB_HIP(hipStreamSynchronize(s));
        }
        for (int q = 0; q < ns; ++q) {
            std::fill(g[q].begin(), g[q].end(), 0.0);
            g[q][0] = beta[q];
            running[q] = active[q];
            nk[q] = 0;
        }
        int j = 0;
        for (; j < m && it < maxit; ++j) {
            double *vj = V + (int64_t)j * n, *zj = Z + (int64_t)j * n, *vn = V + (int64_t)(j + 1) * n;
            precond(vj, zj, nv);
            panel_spmv<double>(A, zj, vn, s, nv);
            seg_dots(sg, kw, n, j + 1, V, vn, h1, ld, s);
            k_seg_update<<<grid_for(n, 256), 256, 0, s>>>(n, sg.rowseg.p, j + 1, V, n, h1, ld, vn);
            VB_LAUNCH_CHECK();
            seg_dots(sg, kw, n, j + 1, V, vn, h2, ld, s);
            k_seg_update<<<grid_for(n, 256), 256, 0, s>>>(n, sg.rowseg.p, j + 1, V, n, h2, ld, vn);
            VB_LAUNCH_CHECK();
            seg_dots(sg, kw, n, 1, vn, vn, hn, ld, s);
            VB_HIP(hipMemcpyAsync(hcopy.data(), kw.hbuf.p, sizeof(double) * 3 * ns * ld, hipMemcpyDeviceToHost, s));
            VB_HIP(hipStreamSynchronize(s));
            std::vector<double> den((size_t)ns * ld, 0.0);
            bool still = false;
            ++it;
            for (int q = 0; q < ns; ++q) {
                if (!running[q]) continue;
                const double *a1 = hcopy.data() + (size_t)q * ld, *a2 = hcopy.data() + (size_t)(ns + q) * ld;
                const double hnorm = std::sqrt(hcopy[(size_t)(2 * ns + q) * ld]);
                den[(size_t)q * ld] = hnorm;
                std::vector<double> &Hq = H[q];
                for (int k = 0; k <= j; ++k) Hq[k * m + j] = a1[k] + a2[k];
                Hq[(j + 1) * m + j] = hnorm;
                for (int k = 0; k < j; ++k) {
                    const double aa = Hq[k * m + j], cc = Hq[(k + 1) * m + j];
                    Hq[k * m + j] = cs[q][k] * aa + sn[q][k] * cc;
                    Hq[(k + 1) * m + j] = -sn[q][k] * aa + cs[q][k] * cc;
                }
                const double aa = Hq[j * m + j], cc = Hq[(j + 1) * m + j];
                const double r = std::sqrt(aa * aa + cc * cc);
                cs[q][j] = r > 0.0 ? aa / r : 1.0;
                sn[q][j] = r > 0.0 ? cc / r : 0.0;
                Hq[j * m + j] = r;
                Hq[(j + 1) * m + j] = 0.0;
                g[q][j + 1] = -sn[q][j] * g[q][j];
                g[q][j] = cs[q][j] * g[q][j];
                nk[q] = j + 1;
                info[q].iters += 1;
                if (!std::isfinite(g[q][j + 1])) fail(VBARMS_ERR_NAN, "Arnoldi produced NaN or Inf");
                if (std::fabs(g[q][j + 1]) <= tol * bn[q] || hnorm == 0.0) running[q] = 0;
                else still = true;
            }
            // v_{j+1} /= ||v_{j+1}|| per running system (others become 0 and are not used)
            to_device(hn, den.data(), (size_t)ns * ld, s);
            upload_active(running);
            k_seg_scale<<<grid_for(n, 256), 256, 0, s>>>(n, sg.rowseg.p, vn, hn, ld, d_active, vn);
            VB_LAUNCH_CHECK();
            VB_HIP(hipStreamSynchronize(s));
            if (!still) {
                ++j;
                break;
            }
        }
        // x += Z y per system, from its own triangular system of nk[q] columns
        std::fill(yall.begin(), yall.end(), 0.0);
        for (int q = 0; q < ns; ++q) {
            const int jq = nk[q];
            double *y = yall.data() + (size_t)q * (m + 1);
            for (int k = jq - 1; k >= 0; --k) {
                double sum = g[q][k];
                for (int c = k + 1; c < jq; ++c) sum -= H[q][k * m + c] * y[c];
                y[k] = sum / H[q][k * m + k];
            }
            if (jq > 0) info[q].restarts += 1;
        }
        to_device(kw.ybuf.p, yall.data(), (size_t)ns * (m + 1), s);
        to_device(d_nk, nk.data(), ns, s);
        k_seg_xupdate<<<grid_for(n, 256), 256, 0, s>>>(n, sg.rowseg.p, d_nk, Z, n, kw.ybuf.p, m + 1, x);
        VB_LAUNCH_CHECK();
        VB_HIP(hipStreamSynchronize(s));  // host vectors above are copy sources
    }
    int worst = VBARMS_OK;
    for (int q = 0; q < ns; ++q)
        if (info[q].status != VBARMS_OK) worst = VBARMS_NOT_CONVERGED;
    for (int q = 0; q < ns; ++q) info[q].fp64_refactor = 0;
    return worst;
}

}  // namespace vb
