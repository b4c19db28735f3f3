// One level of the VBARMS partial block factorization (Sec. 3, Steps 2-4).
//
//   scaling      S1 = 1/max|a| per row, S2 = 1/max|s1 a| per column      (Step 2)
//   independent  natural-order greedy set on the quotient graph of A + A^T (Step 3)
//   pivots       GEPP of every independent diagonal block D_i           (Step 4)
//   G = L^{-1}PF one lane per panel column of an independent block row  (IKJ pass 1)
//   W = E U^{-1} one lane per (row, block) of a remaining block row      (IKJ pass 2)
//   S = C - W G  one workgroup per remaining block row, rows of G streamed in ascending
//                order of the independent block, so each entry sees the same subtraction
//                sequence as the sequential algorithm (Eq. schurl)
// Blocks of G, W and off-diagonal blocks of S are dropped when ||B||_F/(m n) < t.
#include <algorithm>

#include "factor.h"

namespace vb {

namespace {

constexpr int kTG = 8;  // lanes per scalar row in row-streaming kernels

__device__ inline unsigned long long dbits(double x) { return (unsigned long long)__double_as_longlong(x); }

template <class T>
__global__ void k_rowmax(int64_t n, const int *rowblk, const int *rb, const int64_t *wp, const int64_t *vp,
                         const T *v, double *s1) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = gid / kTG;
    int lane = (int)(gid % kTG);
    double mx = 0.0;
    if (row < n) {
        int I = rowblk[row];
        int64_t W = wp[I + 1] - wp[I];
        const T *a = v + vp[I] + (row - rb[I]) * W;
        for (int64_t c = lane; c < W; c += kTG) mx = fmax(mx, (double)fabs(a[c]));
    }
#pragma unroll
    for (int off = kTG / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kTG));
    if (row < n && lane == 0) s1[row] = mx > 0.0 ? 1.0 / mx : 1.0;
}

template <class T>
__global__ void k_colmax(int64_t n, const int *rowblk, const int *rb, const int64_t *wp, const int64_t *vp,
                         const int *sc, const T *v, const double *s1, unsigned long long *cmax) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = gid / kTG;
    int lane = (int)(gid % kTG);
    if (row >= n) return;
    int I = rowblk[row];
    int64_t W = wp[I + 1] - wp[I];
    const T *a = v + vp[I] + (row - rb[I]) * W;
    const int *c = sc + wp[I];
    double sr = s1[row];
    for (int64_t j = lane; j < W; j += kTG) {
        double x = fabs(sr * (double)a[j]);
        if (x > 0.0) atomicMax(&cmax[c[j]], dbits(x));
    }
}

__global__ void k_s2(int64_t n, const unsigned long long *cmax, double *s2) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double m = __longlong_as_double((long long)cmax[j]);
    s2[j] = m > 0.0 ? 1.0 / m : 1.0;
}

template <class T>
__global__ void k_scale(int64_t n, const int *rowblk, const int *rb, const int64_t *wp, const int64_t *vp,
                        const int *sc, const T *v, const double *s1, const double *s2, T *out) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t row = gid / kTG;
    int lane = (int)(gid % kTG);
    if (row >= n) return;
    int I = rowblk[row];
    int64_t W = wp[I + 1] - wp[I];
    int64_t off = vp[I] + (row - rb[I]) * W;
    const int *c = sc + wp[I];
    double sr = s1[row];
    for (int64_t j = lane; j < W; j += kTG) out[off + j] = (T)((sr * (double)v[off + j]) * s2[c[j]]);
}

// transpose of the block pattern (for the quotient graph of A + A^T)
__global__ void k_tcount(int p, const int64_t *rp, const int *ci, int *tcnt) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    for (int64_t k = rp[I]; k < rp[I + 1]; ++k) atomicAdd(&tcnt[ci[k]], 1);
}
__global__ void k_tfill(int p, const int64_t *rp, const int *ci, const int64_t *tptr, int *tfill, int *tlist) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    for (int64_t k = rp[I]; k < rp[I + 1]; ++k) {
        int J = ci[k];
        tlist[tptr[J] + atomicAdd(&tfill[J], 1)] = I;
    }
}

__global__ void k_is_flags(int p, const int *state, const int *rb, int *isf, int *restf, int *issz, int *restsz) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    int in = state[I] == 1;
    int m = rb[I + 1] - rb[I];
    isf[I] = in;
    restf[I] = !in;
    issz[I] = in ? m : 0;
    restsz[I] = in ? 0 : m;
}
__global__ void k_numbering(int p, const int *isf, const int *isidx, const int *restidx, const int *isoff,
                            const int *restoff, int *num, int *is_list, int *rest_list, int *is_rb, int *rest_rb) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    if (isf[I]) {
        int i = isidx[I];
        num[I] = i;
        is_list[i] = I;
        is_rb[i] = isoff[I];
    } else {
        int j = restidx[I];
        num[I] = j;
        rest_list[j] = I;
        rest_rb[j] = restoff[I];
    }
}
__global__ void k_block_sq(int nis, const int *is_list, const int *rb, int64_t *sq) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nis) return;
    int I = is_list[i];
    int m = rb[I + 1] - rb[I];
    sq[i] = (int64_t)m * m;
}

template <class T>
__global__ void k_gepp(int nis, const int *is_list, const int *rb, const int64_t *rp, const int *ci, const int *co,
                       const int64_t *wp, const int64_t *vp, const T *v, const int64_t *dlu_off, const int *is_rb,
                       T *dlu, int *dpiv, double min_ratio, int lvl, int *err) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nis) return;
    int I = is_list[i];
    int m = rb[I + 1] - rb[I];
    int64_t W = wp[I + 1] - wp[I];
    int64_t k = dev_find(ci, rp[I], rp[I + 1], I);
    if (k < 0) { dev_set_error(err, VBARMS_ERR_HIP, 2001, I); return; }
    T *d = dlu + dlu_off[i];
    const T *a = v + vp[I] + co[k];
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) d[r * m + c] = a[r * W + c];
    if (!dev_gepp(m, d, dpiv + is_rb[i])) dev_set_error(err, VBARMS_ERR_SINGULAR, lvl, I);
    else dev_count_illcond<T>(m, d, min_ratio, err);
}

// G = L^{-1} P F: one lane per panel column of an independent block row (F columns only)
template <class T>
__global__ void k_compute_g(int p, int64_t nw, const int64_t *wp, const int64_t *vp, const int *rb, const int *sc,
                            const int *colblk, const int *isf, const int *num, const T *v, const T *dlu,
                            const int64_t *dlu_off, const int *dpiv, const int *is_rb, T *out) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nw) return;
    int I = (int)dev_floor(wp, 0, p + 1, g);
    if (!isf[I]) return;
    int J = colblk[sc[g]];
    if (isf[J]) return;
    int m = rb[I + 1] - rb[I];
    int64_t W = wp[I + 1] - wp[I];
    int64_t c = g - wp[I];
    const T *a = v + vp[I] + c;
    T x[VBARMS_MAX_BLOCK];
    for (int r = 0; r < m; ++r) x[r] = a[r * W];
    int i = num[I];
    dev_lu_fwd<T, T>(m, dlu + dlu_off[i], dpiv + is_rb[i], x);
    T *o = out + vp[I] + c;
    for (int r = 0; r < m; ++r) o[r * W] = x[r];
}

// W = E U^{-1}: one lane per (block, row) of a remaining block row (E blocks only)
template <class T>
__global__ void k_compute_w(int p, int64_t nb, int maxm, const int64_t *rp, const int *ci, const int *co,
                            const int64_t *wp, const int64_t *vp, const int *rb, const int *isf, const int *num,
                            const T *v, const T *dlu, const int64_t *dlu_off, T *out) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t k = gid / maxm;
    int r = (int)(gid % maxm);
    if (k >= nb) return;
    int I = (int)dev_floor(rp, 0, p + 1, k);
    int m = rb[I + 1] - rb[I];
    if (r >= m || isf[I]) return;
    int J = ci[k];
    if (!isf[J]) return;
    int nJ = rb[J + 1] - rb[J];
    int64_t W = wp[I + 1] - wp[I];
    int64_t off = vp[I] + r * W + co[k];
    T e[VBARMS_MAX_BLOCK];
    for (int c = 0; c < nJ; ++c) e[c] = v[off + c];
    dev_row_solve_u<T>(nJ, dlu + dlu_off[num[J]], e, 1);
    for (int c = 0; c < nJ; ++c) out[off + c] = e[c];
}

// keep flags of G (mode 0) or W (mode 1) blocks after the drop test
template <class T>
__global__ void k_keep_gw(int p, int64_t nb, const int64_t *rp, const int *ci, const int *co, const int64_t *wp,
                          const int64_t *vp, const int *rb, const int *isf, const T *vals, double t, int mode,
                          int *keep) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    int I = (int)dev_floor(rp, 0, p + 1, k);
    int J = ci[k];
    bool want = mode == 0 ? (isf[I] && !isf[J]) : (!isf[I] && isf[J]);
    if (!want) { keep[k] = 0; return; }
    int m = rb[I + 1] - rb[I], n = rb[J + 1] - rb[J];
    int64_t W = wp[I + 1] - wp[I];
    keep[k] = !dev_drop<T>(m, n, vals + vp[I] + co[k], W, t);
}

// ---- Schur complement --------------------------------------------------------------
constexpr int kSchurCap = 4096;  // LDS set; at most kSchurCap/2 blocks per Schur row
constexpr int kSymThreads = 64;

__device__ inline void set_insert(int *keys, int *count, int *full, int key) {
    if (*full) return;
    unsigned h = ((unsigned)key * 2654435761u) & (kSchurCap - 1);
    for (;;) {
        int old = atomicCAS(&keys[h], -1, key);
        if (old == -1) {
            if (atomicAdd(count, 1) + 1 >= kSchurCap / 2) *full = 1;
            return;
        }
        if (old == key) return;
        h = (h + 1) & (kSchurCap - 1);
    }
}

// block pattern of S row j = C row j U (union of G rows i over the kept W_ji)
__global__ void __launch_bounds__(kSymThreads) k_schur_sym(const int *rest_list, const int64_t *arp, const int *aci,
                                                           const int *isf, const int *num, const int64_t *wrp,
                                                           const int *wci, const int64_t *grp, const int *gci,
                                                           int64_t *cnt, const int64_t *srp, int *sci, int pass,
                                                           int lvl, int *err) {
    __shared__ int keys[kSchurCap];
    __shared__ int list[kSchurCap / 2 + kSymThreads];
    __shared__ int count, full, n2;
    const int j = blockIdx.x, t = threadIdx.x;
    for (int h = t; h < kSchurCap; h += kSymThreads) keys[h] = -1;
    if (t == 0) { count = 0; full = 0; n2 = 0; }
    __syncthreads();
    const int J = rest_list[j];
    for (int64_t k = arp[J] + t; k < arp[J + 1]; k += kSymThreads) {
        int K = aci[k];
        if (!isf[K]) set_insert(keys, &count, &full, num[K]);
    }
    for (int64_t w = wrp[j]; w < wrp[j + 1]; ++w) {
        int i = wci[w];
        for (int64_t g = grp[i] + t; g < grp[i + 1]; g += kSymThreads) set_insert(keys, &count, &full, gci[g]);
    }
    __syncthreads();
    if (full) {
        if (t == 0) dev_set_error(err, VBARMS_ERR_OOM, lvl, j);
        return;
    }
    if (pass == 0) {
        if (t == 0) cnt[j] = count;
        return;
    }
    for (int h = t; h < kSchurCap; h += kSymThreads) {
        int k = keys[h];
        if (k >= 0) list[atomicAdd(&n2, 1)] = k;
    }
    __syncthreads();
    int nl = n2;
    for (int e = t; e < nl; e += kSymThreads) {
        int key = list[e];
        int rank = 0;
        for (int f = 0; f < nl; ++f) rank += list[f] < key;
        sci[srp[j] + rank] = key;
    }
}

constexpr int kSchurThreads = 256;

// S_j = C_j - sum_i W_ji G_i, one workgroup per remaining block row, S row in global memory
template <class T>
__global__ void __launch_bounds__(kSchurThreads) k_schur_num(
    const int *rest_list, const int *arb, const int64_t *awp, const int64_t *avp, const int *asc, const int *colblk,
    const int *isf, const int *num, const T *av, const int *rest_rb, const int64_t *srp, const int *sci,
    const int *sco, const int64_t *swp, const int64_t *svp, T *sv, const int64_t *wrp, const int *wci, const int *wco,
    const int64_t *wwp, const int64_t *wvp, const T *wv, const int *is_rb, const int64_t *grp, const int *gci,
    const int *gco, const int64_t *gwp, const int64_t *gvp, const T *gv, int *err) {
    const int j = blockIdx.x, t = threadIdx.x;
    const int J = rest_list[j];
    const int m = arb[J + 1] - arb[J];
    const int64_t SW = swp[j + 1] - swp[j];
    T *S = sv + svp[j];
    const int64_t s0 = srp[j], s1 = srp[j + 1];
    for (int64_t e = t; e < m * SW; e += kSchurThreads) S[e] = T(0);
    __syncthreads();
    // C part of row J
    {
        const int64_t AW = awp[J + 1] - awp[J];
        const T *A = av + avp[J];
        for (int64_t c = t; c < AW; c += kSchurThreads) {
            int col = asc[awp[J] + c];
            int K = colblk[col];
            if (isf[K]) continue;
            int Kn = num[K];
            int64_t pos = dev_find(sci, s0, s1, Kn);
            if (pos < 0) { dev_set_error(err, VBARMS_ERR_HIP, 2002, j); continue; }
            int64_t sc = sco[pos] + (col - arb[K]);
            for (int r = 0; r < m; ++r) S[r * SW + sc] = A[r * AW + c];
        }
    }
    __syncthreads();
    // subtract W_ji G_i. for ascending i
    const int64_t WW = wwp[j + 1] - wwp[j];
    const T *Wr = wv + wvp[j];
    for (int64_t w = wrp[j]; w < wrp[j + 1]; ++w) {
        const int i = wci[w];
        const int mi = is_rb[i + 1] - is_rb[i];
        const T *Wb = Wr + wco[w];
        const int64_t GW = gwp[i + 1] - gwp[i];
        const T *Gr = gv + gvp[i];
        for (int64_t c = t; c < GW; c += kSchurThreads) {
            int64_t g = dev_floor32(gco, grp[i], grp[i + 1], (int)c);
            int K = gci[g];
            int64_t pos = dev_find(sci, s0, s1, K);
            if (pos < 0) { dev_set_error(err, VBARMS_ERR_HIP, 2003, j); continue; }
            int64_t sc = sco[pos] + (c - gco[g]);
            for (int r = 0; r < m; ++r) {
                T acc = S[r * SW + sc];
                for (int q = 0; q < mi; ++q) acc = acc - Wb[r * WW + q] * Gr[q * GW + c];
                S[r * SW + sc] = acc;
            }
        }
        __syncthreads();
    }
    (void)rest_rb;
}

template <class T>
__global__ void k_keep_schur(int p, int64_t nb, const int64_t *rp, const int *ci, const int *co, const int64_t *wp,
                             const int64_t *vp, const int *rb, const T *v, double t, int drop_schur, int *keep) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    int I = (int)dev_floor(rp, 0, p + 1, k);
    int J = ci[k];
    if (J == I || !drop_schur) { keep[k] = 1; return; }
    int m = rb[I + 1] - rb[I], n = rb[J + 1] - rb[J];
    keep[k] = !dev_drop<T>(m, n, v + vp[I] + co[k], wp[I + 1] - wp[I], t);
}

}  // namespace

// Weight of every block row for the weighted greedy independent set (Sec. 3, Step 3):
// ||A_II||_F / sum_J ||A_IJ||_F, each block's squares summed row-major and the norms summed
// in ascending block column; 0 for a row without stored blocks.
template <class T>
__global__ void k_is_weights(int p, const int *rb, const int64_t *rp, const int *ci, const int *co,
                             const int64_t *wp, const int64_t *vp, const T *v, double *w) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    const int m = rb[I + 1] - rb[I];
    const int64_t W = wp[I + 1] - wp[I];
    const T *a = v + vp[I];
    double diag = 0.0, tot = 0.0;
    for (int64_t k = rp[I]; k < rp[I + 1]; ++k) {
        const int J = ci[k];
        const int c0 = co[k];
        const int nJ = (k + 1 < rp[I + 1] ? co[k + 1] : (int)W) - c0;
        double ss = 0.0;
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < nJ; ++c) {
                const double x = (double)a[(int64_t)r * W + c0 + c];
                ss = ss + x * x;
            }
        const double f = sqrt(ss);
        tot = tot + f;
        if (J == I) diag = f;
    }
    w[I] = tot > 0.0 ? diag / tot : 0.0;
}

template <class T>
void factor_level(Level<T> &L, Panel<T> &&Ain, int lvl, double droptol, int drop_schur, int is_order,
                  double min_ratio, Panel<T> &next, int *err, hipStream_t s) {
    L.A = std::move(Ain);
    const Panel<T> &A = L.A;
    L.p = A.p;
    L.n = A.h_rb.empty() ? 0 : A.h_rb.back();
    const int p = L.p, n = L.n;
    if (A.maxm > VBARMS_MAX_BLOCK) fail(VBARMS_ERR_OOM, "block larger than VBARMS_MAX_BLOCK");

    // Step 2: scaling
    L.s1.alloc(std::max(n, 1));
    L.s2.alloc(std::max(n, 1));
    {
        DBuf<unsigned long long> cm(std::max(n, 1));
        fill_val<unsigned long long>(cm.p, 0ull, n, s);
        unsigned g = grid_for((int64_t)n * kTG, 256);
        k_rowmax<T><<<g, 256, 0, s>>>(n, A.rowblk.p, A.rb.p, A.wp.p, A.vp.p, A.v.p, L.s1.p);
        VB_LAUNCH_CHECK();
        k_colmax<T><<<g, 256, 0, s>>>(n, A.rowblk.p, A.rb.p, A.wp.p, A.vp.p, A.sc.p, A.v.p, L.s1.p, cm.p);
        VB_LAUNCH_CHECK();
        k_s2<<<grid_for(n, 256), 256, 0, s>>>(n, cm.p, L.s2.p);
        VB_LAUNCH_CHECK();
        // scaled copy shares the layout
        panel_convert<T, T>(A, L.As, s);
        k_scale<T><<<g, 256, 0, s>>>(n, A.rowblk.p, A.rb.p, A.wp.p, A.vp.p, A.sc.p, A.v.p, L.s1.p, L.s2.p, L.As.v.p);
        VB_LAUNCH_CHECK();
    }
    const Panel<T> &As = L.As;

    // Step 3: independent set on the quotient graph of A + A^T, in natural order or by
    // descending weight
    DBuf<int> state(std::max(p, 1));
    DBuf<double> wts;
    if (is_order == 1 && p > 0) {
        wts.alloc(p);
        k_is_weights<T><<<grid_for(p, 256), 256, 0, s>>>(p, As.rb.p, As.rp.p, As.ci.p, As.co.p, As.wp.p, As.vp.p,
                                                         As.v.p, wts.p);
        VB_LAUNCH_CHECK();
    }
    {
        DBuf<int> tcnt(std::max(p, 1)), tfill(std::max(p, 1));
        DBuf<int64_t> tptr(p + 1);
        fill_i32(tcnt.p, 0, p, s);
        fill_i32(tfill.p, 0, p, s);
        if (p > 0) {
            k_tcount<<<grid_for(p, 256), 256, 0, s>>>(p, As.rp.p, As.ci.p, tcnt.p);
            VB_LAUNCH_CHECK();
        }
        int64_t nt = scan_i32_to_i64(tcnt.p, tptr.p, p, s);
        DBuf<int> tlist(std::max<int64_t>(nt, 1));
        if (p > 0) {
            k_tfill<<<grid_for(p, 256), 256, 0, s>>>(p, As.rp.p, As.ci.p, tptr.p, tfill.p, tlist.p);
            VB_LAUNCH_CHECK();
        }
        lfmis(p, As.rp.p, As.ci.p, tptr.p, tlist.p, wts.p, state.p, s);
    }
    // P_I: independent blocks ascending, then the rest ascending
    L.is_flag.alloc(std::max(p, 1));
    L.num.alloc(std::max(p, 1));
    {
        DBuf<int> restf(std::max(p, 1)), issz(std::max(p, 1)), restsz(std::max(p, 1));
        DBuf<int> isidx(p + 1), restidx(p + 1), isoff(p + 1), restoff(p + 1);
        if (p > 0) {
            k_is_flags<<<grid_for(p, 256), 256, 0, s>>>(p, state.p, As.rb.p, L.is_flag.p, restf.p, issz.p, restsz.p);
            VB_LAUNCH_CHECK();
        }
        L.nis = scan_i32(L.is_flag.p, isidx.p, p, s);
        L.nrest = p - L.nis;
        scan_i32(restf.p, restidx.p, p, s, false);
        L.n_is = scan_i32(issz.p, isoff.p, p, s);
        L.n_rest = n - L.n_is;
        scan_i32(restsz.p, restoff.p, p, s, false);
        L.is_list.alloc(std::max(L.nis, 1));
        L.rest_list.alloc(std::max(L.nrest, 1));
        L.is_rb.alloc(L.nis + 1);
        L.rest_rb.alloc(L.nrest + 1);
        if (p > 0) {
            k_numbering<<<grid_for(p, 256), 256, 0, s>>>(p, L.is_flag.p, isidx.p, restidx.p, isoff.p, restoff.p,
                                                          L.num.p, L.is_list.p, L.rest_list.p, L.is_rb.p, L.rest_rb.p);
            VB_LAUNCH_CHECK();
        }
        VB_HIP(hipMemcpyAsync(L.is_rb.p + L.nis, &L.n_is, sizeof(int), hipMemcpyHostToDevice, s));
        VB_HIP(hipMemcpyAsync(L.rest_rb.p + L.nrest, &L.n_rest, sizeof(int), hipMemcpyHostToDevice, s));
        to_host(L.h_is_rb, L.is_rb.p, L.nis + 1, s);
        to_host(L.h_rest_rb, L.rest_rb.p, L.nrest + 1, s);
    }
    const int nis = L.nis, nrest = L.nrest;

    // Step 4: pivot blocks
    L.dlu_off.alloc(nis + 1);
    {
        DBuf<int64_t> sq(std::max(nis, 1));
        if (nis > 0) {
            k_block_sq<<<grid_for(nis, 256), 256, 0, s>>>(nis, L.is_list.p, As.rb.p, sq.p);
            VB_LAUNCH_CHECK();
        }
        int64_t tot = scan_i64(sq.p, L.dlu_off.p, nis, s);
        L.dlu.alloc(std::max<int64_t>(tot, 1));
        L.dpiv.alloc(std::max(L.n_is, 1));
        if (nis > 0) {
            k_gepp<T><<<grid_for(nis, 64), 64, 0, s>>>(nis, L.is_list.p, As.rb.p, As.rp.p, As.ci.p, As.co.p, As.wp.p,
                                                      As.vp.p, As.v.p, L.dlu_off.p, L.is_rb.p, L.dlu.p, L.dpiv.p,
                                                      min_ratio, lvl,
                                                      err);
            VB_LAUNCH_CHECK();
        }
        if (read_one(err, s) != 0) return;
    }

    // G = L^{-1} P F and W = E U^{-1} into one scratch copy (their blocks are disjoint)
    DBuf<T> tmp(std::max<int64_t>(As.nv, 1));
    DBuf<int> keep(std::max<int64_t>(As.nb, 1));
    if (As.nw > 0) {
        k_compute_g<T><<<grid_for(As.nw, 128), 128, 0, s>>>(p, As.nw, As.wp.p, As.vp.p, As.rb.p, As.sc.p,
                                                             As.rowblk.p, L.is_flag.p, L.num.p, As.v.p, L.dlu.p,
                                                             L.dlu_off.p, L.dpiv.p, L.is_rb.p, tmp.p);
        VB_LAUNCH_CHECK();
        k_compute_w<T><<<grid_for(As.nb * As.maxm, 128), 128, 0, s>>>(p, As.nb, As.maxm, As.rp.p, As.ci.p, As.co.p,
                                                                       As.wp.p, As.vp.p, As.rb.p, L.is_flag.p,
                                                                       L.num.p, As.v.p, L.dlu.p, L.dlu_off.p, tmp.p);
        VB_LAUNCH_CHECK();
    }
    if (As.nb > 0) {
        k_keep_gw<T><<<grid_for(As.nb, 256), 256, 0, s>>>(p, As.nb, As.rp.p, As.ci.p, As.co.p, As.wp.p, As.vp.p,
                                                           As.rb.p, L.is_flag.p, tmp.p, droptol, 0, keep.p);
        VB_LAUNCH_CHECK();
    }
    panel_compact<T>(As, tmp.p, keep.p, L.is_list.p, nis, L.num.p, L.h_is_rb, L.h_rest_rb, L.G, s);
    if (As.nb > 0) {
        k_keep_gw<T><<<grid_for(As.nb, 256), 256, 0, s>>>(p, As.nb, As.rp.p, As.ci.p, As.co.p, As.wp.p, As.vp.p,
                                                           As.rb.p, L.is_flag.p, tmp.p, droptol, 1, keep.p);
        VB_LAUNCH_CHECK();
    }
    panel_compact<T>(As, tmp.p, keep.p, L.rest_list.p, nrest, L.num.p, L.h_rest_rb, L.h_is_rb, L.W, s);
    tmp.release();

    // Schur complement: symbolic, numeric, drop, compact
    Panel<T> S;
    panel_set_blocks(S, L.h_rest_rb, L.h_rest_rb, s);
    S.rp.alloc(nrest + 1);
    {
        DBuf<int64_t> cnt(std::max(nrest, 1));
        if (nrest > 0) {
            k_schur_sym<<<nrest, kSymThreads, 0, s>>>(L.rest_list.p, As.rp.p, As.ci.p, L.is_flag.p, L.num.p, L.W.rp.p,
                                                      L.W.ci.p, L.G.rp.p, L.G.ci.p, cnt.p, nullptr, nullptr, 0, lvl,
                                                      err);
            VB_LAUNCH_CHECK();
        }
        if (read_one(err, s) != 0) return;
        S.nb = scan_i64(cnt.p, S.rp.p, nrest, s);
        S.ci.alloc(std::max<int64_t>(S.nb, 1));
        if (nrest > 0) {
            k_schur_sym<<<nrest, kSymThreads, 0, s>>>(L.rest_list.p, As.rp.p, As.ci.p, L.is_flag.p, L.num.p, L.W.rp.p,
                                                      L.W.ci.p, L.G.rp.p, L.G.ci.p, cnt.p, S.rp.p, S.ci.p, 1, lvl,
                                                      err);
            VB_LAUNCH_CHECK();
        }
    }
    panel_finish_layout(S, s);
    S.v.alloc(std::max<int64_t>(S.nv, 1));
    if (nrest > 0) {
        k_schur_num<T><<<nrest, kSchurThreads, 0, s>>>(
            L.rest_list.p, As.rb.p, As.wp.p, As.vp.p, As.sc.p, As.rowblk.p, L.is_flag.p, L.num.p, As.v.p, L.rest_rb.p,
            S.rp.p, S.ci.p, S.co.p, S.wp.p, S.vp.p, S.v.p, L.W.rp.p, L.W.ci.p, L.W.co.p, L.W.wp.p, L.W.vp.p, L.W.v.p,
            L.is_rb.p, L.G.rp.p, L.G.ci.p, L.G.co.p, L.G.wp.p, L.G.vp.p, L.G.v.p, err);
        VB_LAUNCH_CHECK();
    }
    DBuf<int> skeep(std::max<int64_t>(S.nb, 1));
    if (S.nb > 0) {
        k_keep_schur<T><<<grid_for(S.nb, 256), 256, 0, s>>>(nrest, S.nb, S.rp.p, S.ci.p, S.co.p, S.wp.p, S.vp.p,
                                                             S.rb.p, S.v.p, droptol, drop_schur, skeep.p);
        VB_LAUNCH_CHECK();
    }
    panel_compact<T>(S, nullptr, skeep.p, nullptr, nrest, nullptr, L.h_rest_rb, L.h_rest_rb, next, s);
    L.y.alloc(std::max(L.n_is, 1));
    L.t.alloc(std::max(L.n_is, 1));
}

template void factor_level<double>(Level<double> &, Panel<double> &&, int, double, int, int, double, Panel<double> &,
                                   int *, hipStream_t);
template void factor_level<float>(Level<float> &, Panel<float> &&, int, double, int, int, double, Panel<float> &, int *,
                                  hipStream_t);

}  // namespace vb
