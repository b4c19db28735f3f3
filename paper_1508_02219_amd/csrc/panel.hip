// Block-row panel layout: construction from CSR (Eq. blockperm), compaction after
// dropping, and export in block-sparse-row form.
#include "common.h"

namespace vb {

namespace {

// per block row: panel column offsets of its blocks and its width
__global__ void k_row_layout(int p, const int *rb, const int *cb, const int64_t *rp, const int *ci, int *co,
                             int64_t *width, int64_t *area) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    int acc = 0;
    for (int64_t k = rp[I]; k < rp[I + 1]; ++k) {
        co[k] = acc;
        int J = ci[k];
        acc += cb[J + 1] - cb[J];
    }
    width[I] = acc;
    area[I] = (int64_t)acc * (rb[I + 1] - rb[I]);
}

// scalar column list of every panel, one thread per block
__global__ void k_row_sc(int p, int64_t nb, const int *cb, const int64_t *rp, const int *ci, const int *co,
                         const int64_t *wp, int *sc) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const int I = (int)dev_floor(rp, 0, p + 1, k);
    const int J = ci[k];
    int *d = sc + wp[I] + co[k];
    for (int c = cb[J]; c < cb[J + 1]; ++c) *d++ = c;
}

// ---- CSR -> panel ----------------------------------------------------------------
constexpr int kSymCap = 4096;  // LDS hash capacity; at most kSymCap/2 distinct block columns
constexpr int kSymThreads = 64;

__device__ inline bool lds_set_insert(int *keys, int *count, int *full, int key) {
    if (*full) return false;
    unsigned h = ((unsigned)key * 2654435761u) & (kSymCap - 1);
    for (;;) {
        int old = atomicCAS(&keys[h], -1, key);
        if (old == -1) {
            int c = atomicAdd(count, 1);
            if (c + 1 >= kSymCap / 2) *full = 1;
            return true;
        }
        if (old == key) return false;
        h = (h + 1) & (kSymCap - 1);
    }
}

// pass 0: count distinct block columns of every block row; pass 1: write them sorted
__global__ void __launch_bounds__(kSymThreads) k_vbsr_sym(const int64_t *rowptr, const int *col, const int *perm,
                                                          const int *inv, const int *blkof, const int *bptr,
                                                          int64_t *cnt, const int64_t *rp, int *ci, int pass,
                                                          int *err) {
    __shared__ int keys[kSymCap];
    __shared__ int list[kSymCap / 2 + kSymThreads];
    __shared__ int count, full;
    const int I = blockIdx.x;
    const int t = threadIdx.x;
    for (int h = t; h < kSymCap; h += kSymThreads) keys[h] = -1;
    if (t == 0) { count = 0; full = 0; }
    __syncthreads();
    if (t == 0) lds_set_insert(keys, &count, &full, I);
    for (int r = bptr[I]; r < bptr[I + 1]; ++r) {
        int orow = perm[r];
        for (int64_t k = rowptr[orow] + t; k < rowptr[orow + 1]; k += kSymThreads)
            lds_set_insert(keys, &count, &full, blkof[inv[col[k]]]);
    }
    __syncthreads();
    if (full) {
        if (t == 0) dev_set_error(err, VBARMS_ERR_OOM, I, kSymCap / 2);
        return;
    }
    if (pass == 0) {
        if (t == 0) cnt[I] = count;
        return;
    }
    __shared__ int n2;
    if (t == 0) n2 = 0;
    __syncthreads();
    for (int h = t; h < kSymCap; h += kSymThreads) {
        int k = keys[h];
        if (k >= 0) list[atomicAdd(&n2, 1)] = k;
    }
    __syncthreads();
    int nl = n2;
    int64_t base = rp[I];
    for (int e = t; e < nl; e += kSymThreads) {
        int key = list[e];
        int rank = 0;
        for (int f = 0; f < nl; ++f) rank += list[f] < key;
        ci[base + rank] = key;
    }
}

__global__ void k_inv_perm(const int *perm, int *inv, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[perm[i]] = i;
}

__global__ void k_vbsr_num(int n, const int64_t *rowptr, const int *col, const double *val, const int *inv,
                           const int *blkof, const int *bptr, const int64_t *rp, const int *ci, const int *co,
                           const int64_t *wp, const int64_t *vp, double *v, int *err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int r = inv[i];
    int I = blkof[r];
    int rl = r - bptr[I];
    int64_t W = wp[I + 1] - wp[I];
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        double a = val[k];
        if (!isfinite(a)) dev_set_error(err, VBARMS_ERR_NAN, i, (int)(k - rowptr[i]));
        int c = inv[col[k]];
        int J = blkof[c];
        int64_t pos = dev_find(ci, rp[I], rp[I + 1], J);
        if (pos < 0) { dev_set_error(err, VBARMS_ERR_HIP, 2004, i); continue; }
        v[vp[I] + rl * W + co[pos] + (c - bptr[J])] = a;
    }
}

// ---- compaction -------------------------------------------------------------------
__global__ void k_compact_count(int dst_p, const int *src_row_of, const int64_t *srp, const int *keep,
                                int64_t *cnt) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= dst_p) return;
    int sr = src_row_of ? src_row_of[r] : r;
    int64_t c = 0;
    for (int64_t k = srp[sr]; k < srp[sr + 1]; ++k) c += keep ? (keep[k] != 0) : 1;
    cnt[r] = c;
}
__global__ void k_compact_cols(int dst_p, const int *src_row_of, const int64_t *srp, const int *sci,
                               const int *keep, const int *newcol, const int64_t *drp, int *dci, int64_t *srck) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= dst_p) return;
    int sr = src_row_of ? src_row_of[r] : r;
    int64_t d = drp[r];
    for (int64_t k = srp[sr]; k < srp[sr + 1]; ++k) {
        if (keep && !keep[k]) continue;
        dci[d] = newcol ? newcol[sci[k]] : sci[k];
        srck[d] = k;
        ++d;
    }
}
// source panel column of every destination panel column
__global__ void k_compact_srcpc(int dst_p, const int *dcb, const int64_t *drp, const int *dci, const int *dco,
                                const int64_t *dwp, const int64_t *srck, const int *sco, int *srcpc) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= dst_p) return;
    for (int64_t k = drp[r]; k < drp[r + 1]; ++k) {
        int J = dci[k];
        int nJ = dcb[J + 1] - dcb[J];
        int s0 = sco[srck[k]];
        int64_t d0 = dwp[r] + dco[k];
        for (int c = 0; c < nJ; ++c) srcpc[d0 + c] = s0 + c;
    }
}
// one thread per (destination scalar row, panel column chunk)
template <class T>
__global__ void k_compact_vals(int64_t nrows, const int *drowblk, const int *drb, const int *src_row_of,
                               const int *srb, const int64_t *swp, const int64_t *svp, const T *sv,
                               const int64_t *dwp, const int64_t *dvp, const int *srcpc, T *dv) {
    constexpr int G = 16;
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = gid / G;
    int lane = (int)(gid % G);
    if (row >= nrows) return;
    int I = drowblk[row];
    int rl = (int)(row - drb[I]);
    int sr = src_row_of ? src_row_of[I] : I;
    int64_t W = dwp[I + 1] - dwp[I];
    int64_t SW = swp[sr + 1] - swp[sr];
    const T *s = sv + svp[sr] + rl * SW;
    T *d = dv + dvp[I] + rl * W;
    const int *pc = srcpc + dwp[I];
    for (int64_t c = lane; c < W; c += G) d[c] = s[pc[c]];
}

template <class T>
__global__ void k_export_vals(int p, const int *rb, const int *cb, const int64_t *rp, const int *ci,
                              const int *co, const int64_t *wp, const int64_t *vp, const int64_t *boff,
                              const T *v, double *out) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    int m = rb[I + 1] - rb[I];
    int64_t W = wp[I + 1] - wp[I];
    for (int64_t k = rp[I]; k < rp[I + 1]; ++k) {
        int J = ci[k];
        int n = cb[J + 1] - cb[J];
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < n; ++c) out[boff[k] + r * n + c] = (double)v[vp[I] + r * W + co[k] + c];
    }
}
__global__ void k_block_area(int p, const int *rb, const int *cb, const int64_t *rp, const int *ci, int64_t *area) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    int m = rb[I + 1] - rb[I];
    for (int64_t k = rp[I]; k < rp[I + 1]; ++k) area[k] = (int64_t)m * (cb[ci[k] + 1] - cb[ci[k]]);
}

}  // namespace

template <class T>
void panel_set_blocks(Panel<T> &a, const std::vector<int> &rb, const std::vector<int> &cb, hipStream_t s) {
    a.p = (int)rb.size() - 1;
    a.q = (int)cb.size() - 1;
    a.h_rb = rb;
    a.h_cb = cb;
    a.rb.alloc(rb.size());
    a.cb.alloc(cb.size());
    to_device(a.rb.p, rb.data(), rb.size(), s);
    to_device(a.cb.p, cb.data(), cb.size(), s);
    a.maxm = 0;
    for (int i = 0; i < a.p; ++i) a.maxm = std::max(a.maxm, rb[i + 1] - rb[i]);
    a.rowblk.alloc(std::max(rb.back(), 1));
    fill_rowblk(a.rb.p, a.p, a.rowblk.p, s);
}

template <class T>
void panel_finish_layout(Panel<T> &a, hipStream_t s) {
    a.co.alloc(std::max<int64_t>(a.nb, 1));
    a.wp.alloc(a.p + 1);
    a.vp.alloc(a.p + 1);
    DBuf<int64_t> width(std::max(a.p, 1)), area(std::max(a.p, 1));
    if (a.p > 0) {
        k_row_layout<<<grid_for(a.p, 256), 256, 0, s>>>(a.p, a.rb.p, a.cb.p, a.rp.p, a.ci.p, a.co.p, width.p, area.p);
        VB_LAUNCH_CHECK();
    }
    a.nw = scan_i64(width.p, a.wp.p, a.p, s);
    a.nv = scan_i64(area.p, a.vp.p, a.p, s);
    a.sc.alloc(std::max<int64_t>(a.nw, 1));
    if (a.nb > 0) {
        k_row_sc<<<grid_for(a.nb, 256), 256, 0, s>>>(a.p, a.nb, a.cb.p, a.rp.p, a.ci.p, a.co.p, a.wp.p, a.sc.p);
        VB_LAUNCH_CHECK();
    }
}

template <class T>
void panel_compact(const Panel<T> &src, const T *vals, const int *keep, const int *src_row_of, int dst_p, const int *newcol,
                   const std::vector<int> &dst_rb, const std::vector<int> &dst_cb, Panel<T> &dst, hipStream_t s) {
    panel_set_blocks(dst, dst_rb, dst_cb, s);
    dst.rp.alloc(dst_p + 1);
    DBuf<int64_t> cnt(std::max(dst_p, 1));
    if (dst_p > 0) {
        k_compact_count<<<grid_for(dst_p, 256), 256, 0, s>>>(dst_p, src_row_of, src.rp.p, keep, cnt.p);
        VB_LAUNCH_CHECK();
    }
    dst.nb = scan_i64(cnt.p, dst.rp.p, dst_p, s);
    dst.ci.alloc(std::max<int64_t>(dst.nb, 1));
    DBuf<int64_t> srck(std::max<int64_t>(dst.nb, 1));
    if (dst_p > 0) {
        k_compact_cols<<<grid_for(dst_p, 256), 256, 0, s>>>(dst_p, src_row_of, src.rp.p, src.ci.p, keep, newcol,
                                                            dst.rp.p, dst.ci.p, srck.p);
        VB_LAUNCH_CHECK();
    }
    panel_finish_layout(dst, s);
    dst.v.alloc(std::max<int64_t>(dst.nv, 1));
    if (dst.nb == 0 || dst_p == 0) return;
    DBuf<int> srcpc(std::max<int64_t>(dst.nw, 1));
    k_compact_srcpc<<<grid_for(dst_p, 256), 256, 0, s>>>(dst_p, dst.cb.p, dst.rp.p, dst.ci.p, dst.co.p, dst.wp.p,
                                                         srck.p, src.co.p, srcpc.p);
    VB_LAUNCH_CHECK();
    int64_t nrows = dst_rb.back();
    k_compact_vals<T><<<grid_for(nrows * 16, 256), 256, 0, s>>>(nrows, dst.rowblk.p, dst.rb.p, src_row_of, src.rb.p,
                                                                 src.wp.p, src.vp.p, vals ? vals : src.v.p, dst.wp.p, dst.vp.p,
                                                                 srcpc.p, dst.v.p);
    VB_LAUNCH_CHECK();
}

template <class T>
void panel_export(const Panel<T> &a, std::vector<int64_t> &rowptr, std::vector<int> &colidx, std::vector<double> &vals,
                  hipStream_t s) {
    to_host(rowptr, a.rp.p, a.p + 1, s);
    to_host(colidx, a.ci.p, a.nb, s);
    DBuf<int64_t> area(std::max<int64_t>(a.nb, 1)), boff(a.nb + 1);
    if (a.p > 0) {
        k_block_area<<<grid_for(a.p, 256), 256, 0, s>>>(a.p, a.rb.p, a.cb.p, a.rp.p, a.ci.p, area.p);
        VB_LAUNCH_CHECK();
    }
    int64_t total = scan_i64(area.p, boff.p, a.nb, s);
    DBuf<double> out(std::max<int64_t>(total, 1));
    if (a.p > 0) {
        k_export_vals<T><<<grid_for(a.p, 64), 64, 0, s>>>(a.p, a.rb.p, a.cb.p, a.rp.p, a.ci.p, a.co.p, a.wp.p, a.vp.p,
                                                         boff.p, a.v.p, out.p);
        VB_LAUNCH_CHECK();
    }
    to_host(vals, out.p, total, s);
}

template <class Tin, class Tout>
__global__ void k_convert(const Tin *a, Tout *b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (Tout)a[i];
}

template <class T>
static void copy_dev(DBuf<T> &dst, const DBuf<T> &src, size_t n, hipStream_t s) {
    dst.alloc(std::max<size_t>(n, 1));
    if (n) VB_HIP(hipMemcpyAsync(dst.p, src.p, n * sizeof(T), hipMemcpyDeviceToDevice, s));
}

// Same layout, values converted to Tout.
template <class Tin, class Tout>
void panel_convert(const Panel<Tin> &a, Panel<Tout> &b, hipStream_t s) {
    b.p = a.p; b.q = a.q; b.nb = a.nb; b.nw = a.nw; b.nv = a.nv; b.maxm = a.maxm;
    b.h_rb = a.h_rb; b.h_cb = a.h_cb;
    copy_dev(b.rb, a.rb, a.p + 1, s);
    copy_dev(b.cb, a.cb, a.q + 1, s);
    copy_dev(b.rp, a.rp, a.p + 1, s);
    copy_dev(b.wp, a.wp, a.p + 1, s);
    copy_dev(b.vp, a.vp, a.p + 1, s);
    copy_dev(b.ci, a.ci, a.nb, s);
    copy_dev(b.co, a.co, a.nb, s);
    copy_dev(b.sc, a.sc, a.nw, s);
    copy_dev(b.rowblk, a.rowblk, a.h_rb.empty() ? 0 : a.h_rb.back(), s);
    b.v.alloc(std::max<int64_t>(a.nv, 1));
    if (a.nv) {
        k_convert<Tin, Tout><<<grid_for(a.nv, 256), 256, 0, s>>>(a.v.p, b.v.p, a.nv);
        VB_LAUNCH_CHECK();
    }
}
template void panel_convert<double, double>(const Panel<double> &, Panel<double> &, hipStream_t);
template void panel_convert<double, float>(const Panel<double> &, Panel<float> &, hipStream_t);
template void panel_convert<float, float>(const Panel<float> &, Panel<float> &, hipStream_t);

// Builds P_B A P_B^T in panel form.  Every block row carries its diagonal block.
void panel_from_csr(int n, const int64_t *rowptr, const int *col, const double *val, const int *perm,
                    const std::vector<int> &bptr, Panel<double> &out, int *err, hipStream_t s) {
    int p = (int)bptr.size() - 1;
    panel_set_blocks(out, bptr, bptr, s);
    DBuf<int> inv(std::max(n, 1));
    if (n > 0) {
        k_inv_perm<<<grid_for(n, 256), 256, 0, s>>>(perm, inv.p, n);
        VB_LAUNCH_CHECK();
    }
    DBuf<int64_t> cnt(std::max(p, 1));
    out.rp.alloc(p + 1);
    if (p > 0) {
        k_vbsr_sym<<<p, kSymThreads, 0, s>>>(rowptr, col, perm, inv.p, out.rowblk.p, out.rb.p, cnt.p, nullptr,
                                             nullptr, 0, err);
        VB_LAUNCH_CHECK();
    }
    int herr = read_one(err, s);
    if (herr) fail(VBARMS_ERR_OOM, "a block row has more than 2048 distinct block columns");
    out.nb = scan_i64(cnt.p, out.rp.p, p, s);
    out.ci.alloc(std::max<int64_t>(out.nb, 1));
    if (p > 0) {
        k_vbsr_sym<<<p, kSymThreads, 0, s>>>(rowptr, col, perm, inv.p, out.rowblk.p, out.rb.p, cnt.p, out.rp.p,
                                             out.ci.p, 1, err);
        VB_LAUNCH_CHECK();
    }
    panel_finish_layout(out, s);
    out.v.alloc(std::max<int64_t>(out.nv, 1));
    fill_val<double>(out.v.p, 0.0, out.nv, s);
    if (n > 0) {
        k_vbsr_num<<<grid_for(n, 128), 128, 0, s>>>(n, rowptr, col, val, inv.p, out.rowblk.p, out.rb.p, out.rp.p,
                                                    out.ci.p, out.co.p, out.wp.p, out.vp.p, out.v.p, err);
        VB_LAUNCH_CHECK();
    }
}

template void panel_set_blocks<double>(Panel<double> &, const std::vector<int> &, const std::vector<int> &, hipStream_t);
template void panel_set_blocks<float>(Panel<float> &, const std::vector<int> &, const std::vector<int> &, hipStream_t);
template void panel_finish_layout<double>(Panel<double> &, hipStream_t);
template void panel_finish_layout<float>(Panel<float> &, hipStream_t);
template void panel_compact<double>(const Panel<double> &, const double *, const int *, const int *, int, const int *,
                                    const std::vector<int> &, const std::vector<int> &, Panel<double> &, hipStream_t);
template void panel_compact<float>(const Panel<float> &, const float *, const int *, const int *, int, const int *,
                                   const std::vector<int> &, const std::vector<int> &, Panel<float> &, hipStream_t);
template void panel_export<double>(const Panel<double> &, std::vector<int64_t> &, std::vector<int> &,
                                   std::vector<double> &, hipStream_t);
template void panel_export<float>(const Panel<float> &, std::vector<int64_t> &, std::vector<int> &,
                                  std::vector<double> &, hipStream_t);

}  // namespace vb
