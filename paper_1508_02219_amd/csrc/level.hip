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

// Column maxima of |s1_r a_rj|: kTG lanes per block row stride over its panel columns, each
// lane takes the maximum over the block row's scalar rows itself and issues one atomic per
// column of the block row (the maximum does not depend on the order of the rows).
template <class T>
__global__ void k_colmax(int p, const int *rb, const int64_t *wp, const int64_t *vp, const int *sc, const T *v,
                         const double *s1, unsigned long long *cmax) {
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t I = gid / kTG;
    int lane = (int)(gid % kTG);
    if (I >= p) return;
    const int r0 = rb[I], m = rb[I + 1] - r0;
    const int64_t W = wp[I + 1] - wp[I];
    const T *a = v + vp[I];
    const int *c = sc + wp[I];
    for (int64_t j = lane; j < W; j += kTG) {
        double x = 0.0;
        for (int r = 0; r < m; ++r) x = fmax(x, fabs(s1[r0 + r] * (double)a[(int64_t)r * W + j]));
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

// Pivot-block GEPP, one wavefront per block of the independent set (four per workgroup),
// the block staged in LDS and factored by wave_gepp (the same factors as dev_gepp, bit for
// bit).
template <class T>
__global__ void __launch_bounds__(256) k_gepp(int nis, const int *is_list, const int *rb, const int64_t *rp,
                                              const int *ci, const int *co, const int64_t *wp, const int64_t *vp,
                                              const T *v, const int64_t *dlu_off, const int *is_rb, T *dlu,
                                              int *dpiv, int *dperm, double min_ratio, int lvl, int *err) {
    __shared__ T sa[4][VBARMS_MAX_BLOCK * VBARMS_MAX_BLOCK];
    __shared__ int spiv[4][VBARMS_MAX_BLOCK];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + w;
    if (i >= nis) return;  // the whole wavefront leaves; nothing below syncs the workgroup
    const int I = is_list[i];
    const int m = rb[I + 1] - rb[I];
    const int64_t W = wp[I + 1] - wp[I];
    const int64_t k0 = dev_find(ci, rp[I], rp[I + 1], I);
    if (k0 < 0) {
        if (lane == 0) dev_set_error(err, VBARMS_ERR_HIP, 2001, I);
        return;
    }
    T *a = sa[w];
    int *pv = spiv[w];
    const T *src = v + vp[I] + co[k0];
    for (int e = lane; e < m * m; e += 64) a[e] = src[(int64_t)(e / m) * W + (e % m)];
    wave_sync();
    if (!wave_gepp<T>(m, a, pv, lane)) {
        if (lane == 0) dev_set_error(err, VBARMS_ERR_SINGULAR, lvl, I);
        return;
    }
    T *d = dlu + dlu_off[i];
    for (int e = lane; e < m * m; e += 64) d[e] = a[e];
    if (lane < m) dpiv[is_rb[i] + lane] = pv[lane];
    if (lane == 0) {
        dev_count_illcond<T>(m, a, min_ratio, err);
        // the row exchanges as one permutation: row r of P x is row dperm[r] of x
        int *pm = dperm + is_rb[i];
        for (int r = 0; r < m; ++r) pm[r] = r;
        for (int r = 0; r < m; ++r) {
            const int t = pm[r];
            pm[r] = pm[pv[r]];
            pm[pv[r]] = t;
        }
    }
}

// G = L^{-1} P F: one lane per panel column of an independent block row (F columns only)
template <class T>
__global__ void __launch_bounds__(128) k_compute_g(int p, int64_t nw, const int64_t *wp, const int64_t *vp, const int *rb, const int *sc,
                            const int *colblk, const int *isf, const int *num, const T *v, const T *dlu,
                            const int64_t *dlu_off, const int *dperm, const int *is_rb, T *out) {
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
    const int i = num[I];
    const int *pm = dperm + is_rb[i];
    T x[VBARMS_MAX_BLOCK];  // P applied while loading
#pragma unroll
    for (int r = 0; r < VBARMS_MAX_BLOCK; ++r) x[r] = r < m ? a[(int64_t)pm[r] * W] : T(0);
    reg_l_fwd<T, T, VBARMS_MAX_BLOCK>(m, dlu + dlu_off[i], x);
    T *o = out + vp[I] + c;
#pragma unroll
    for (int r = 0; r < VBARMS_MAX_BLOCK; ++r)
        if (r < m) o[r * W] = x[r];
}

// e <- e U^{-1} for a row of up to MAXM entries held in registers: the loops are unrolled
// to MAXM with guards, so the row never leaves registers; the operations and their order
// are those of dev_row_solve_u.
template <class T, int MAXM>
__device__ inline void reg_row_solve_u(int m, const T *lu, T (&e)[MAXM]) {
#pragma unroll
    for (int c = 0; c < MAXM; ++c) {
        if (c < m) {
            T s = e[c];
#pragma unroll
            for (int q = 0; q < c; ++q) s = s - e[q] * lu[q * m + c];
            e[c] = s / lu[c * m + c];
        }
    }
}

// W = E U^{-1}: one lane per scalar row of a remaining block row, its E blocks in turn
template <class T>
__global__ void __launch_bounds__(128) k_compute_w(int n, const int *rowblk, const int64_t *rp, const int *ci, const int *co,
                            const int64_t *wp, const int64_t *vp, const int *rb, const int *isf, const int *num,
                            const T *v, const T *dlu, const int64_t *dlu_off, T *out) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    const int I = rowblk[row];
    if (isf[I]) return;
    const int r = row - rb[I];
    const int64_t W = wp[I + 1] - wp[I];
    for (int64_t k = rp[I]; k < rp[I + 1]; ++k) {
        const int J = ci[k];
        if (!isf[J]) continue;
        const int nJ = rb[J + 1] - rb[J];
        const int64_t off = vp[I] + r * W + co[k];
        T e[VBARMS_MAX_BLOCK];
#pragma unroll
        for (int c = 0; c < VBARMS_MAX_BLOCK; ++c) e[c] = c < nJ ? v[off + c] : T(0);
        reg_row_solve_u<T, VBARMS_MAX_BLOCK>(nJ, dlu + dlu_off[num[J]], e);
#pragma unroll
        for (int c = 0; c < VBARMS_MAX_BLOCK; ++c)
            if (c < nJ) out[off + c] = e[c];
    }
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

namespace {

// ---- groups of supernodes (several supernodes per pivot block) ---------------------
// Step 3 with groups: an unmarked supernode opens a group, its unmarked quotient-graph
// neighbours (A + A^T) join in ascending order while the group keeps at most gmax rows
// (one that does not fit is skipped), then the members and all their neighbours are
// marked.  Every opening depends on all earlier marks, so the greedy is sequential by
// definition; it runs on the host over a copy of the block pattern (p + nb integers).
// Groups are numbered by their smallest supernode, members ascending.
struct HostGroups {
    int ng = 0;
    std::vector<int> gid;            // [p] group, or -1
    std::vector<int> gptr, members;  // members of group g: members[gptr[g] .. gptr[g+1])
};

// In-place ascending sort of a short list by one thread (Shell sort, gaps 701 .. 1); the
// lists here hold tens to a few hundred entries.
__device__ inline void dev_shell_sort(int *c, int64_t k) {
    const int gaps[8] = {701, 301, 132, 57, 23, 10, 4, 1};
    for (int gi = 0; gi < 8; ++gi) {
        const int64_t gap = gaps[gi];
        for (int64_t i = gap; i < k; ++i) {
            const int v = c[i];
            int64_t j = i;
            while (j >= gap && c[j - gap] > v) {
                c[j] = c[j - gap];
                j -= gap;
            }
            c[j] = v;
        }
    }
}

// Neighbour lists of the quotient graph of A + A^T, ascending and without the vertex
// itself: the row list merged with the (sorted) column list.  Pass 0 counts, pass 1 writes.
__global__ void k_sym_adj(int p, const int64_t *rp, const int *ci, const int64_t *tptr, int *tlist, int pass,
                          int64_t *cnt, const int64_t *aptr, int *adj) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= p) return;
    int *t = tlist + tptr[v];
    const int64_t nt = tptr[v + 1] - tptr[v];
    if (pass == 0) dev_shell_sort(t, nt);  // the column list was filled in arbitrary order
    int64_t a = rp[v], ae = rp[v + 1], b = 0, c = 0;
    int last = -1;
    while (a < ae || b < nt) {
        int x;
        if (b >= nt || (a < ae && ci[a] <= t[b])) x = ci[a++];
        else x = t[b++];
        if (x == v || x == last) continue;
        last = x;
        if (pass == 1) adj[aptr[v] + c] = x;
        ++c;
    }
    if (pass == 0) cnt[v] = c;
}

HostGroups host_groups(int p, const int64_t *ap, const int *adj, const std::vector<int> &rb, int gmax,
                       const std::vector<double> *wts) {
    std::vector<int> order(p);
    for (int I = 0; I < p; ++I) order[I] = I;
    if (wts) std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return (*wts)[a] > (*wts)[b]; });
    HostGroups G;
    G.gid.assign(p, -1);
    std::vector<char> marked(p, 0);
    std::vector<int> mem;
    for (int v : order) {
        if (marked[v]) continue;
        const int g = G.ng++;
        int rows = rb[v + 1] - rb[v];
        G.gid[v] = g;
        marked[v] = 1;
        mem.assign(1, v);
        for (int64_t a = ap[v]; a < ap[v + 1]; ++a) {  // neighbours ascending
            const int u = adj[a];
            if (marked[u]) continue;
            const int su = rb[u + 1] - rb[u];
            if (rows + su > gmax) continue;
            G.gid[u] = g;
            marked[u] = 1;
            mem.push_back(u);
            rows += su;
        }
        for (int w : mem)
            for (int64_t a = ap[w]; a < ap[w + 1]; ++a) marked[adj[a]] = 1;
    }
    std::vector<int> renum(G.ng, -1);
    int seen = 0;
    for (int I = 0; I < p; ++I)
        if (G.gid[I] >= 0 && renum[G.gid[I]] < 0) renum[G.gid[I]] = seen++;
    G.gptr.assign(G.ng + 1, 0);
    for (int I = 0; I < p; ++I)
        if (G.gid[I] >= 0) {
            G.gid[I] = renum[G.gid[I]];
            G.gptr[G.gid[I] + 1]++;
        }
    for (int g = 0; g < G.ng; ++g) G.gptr[g + 1] += G.gptr[g];
    G.members.resize(G.gptr[G.ng]);
    std::vector<int> fill(G.gptr.begin(), G.gptr.end() - 1);
    for (int I = 0; I < p; ++I)
        if (G.gid[I] >= 0) G.members[fill[G.gid[I]]++] = I;
    return G;
}

// Neighbour lists of the quotient graph of the pattern of P (A + A^T), built on the device
// and copied to pinned host memory; `ready` is recorded after the copies (the caller waits
// on it).  hap[p+1] and hadj[...] stay valid until the thread's next pinned_staging call.
template <class T>
void sym_adjacency_to_host(const Panel<T> &P, hipStream_t s, hipEvent_t ready, const int64_t *&hap,
                           const int *&hadj) {
    const int p = P.p;
    DBuf<int> tcnt(std::max(p, 1)), tfill(std::max(p, 1));
    DBuf<int64_t> tptr(p + 1), acnt(std::max(p, 1)), aptr(p + 1);
    fill_i32(tcnt.p, 0, p, s);
    fill_i32(tfill.p, 0, p, s);
    if (p > 0) {
        k_tcount<<<grid_for(p, 256), 256, 0, s>>>(p, P.rp.p, P.ci.p, tcnt.p);
        VB_LAUNCH_CHECK();
    }
    const int64_t nt = scan_i32_to_i64(tcnt.p, tptr.p, p, s);
    DBuf<int> tlist(std::max<int64_t>(nt, 1));
    if (p > 0) {
        k_tfill<<<grid_for(p, 256), 256, 0, s>>>(p, P.rp.p, P.ci.p, tptr.p, tfill.p, tlist.p);
        VB_LAUNCH_CHECK();
        k_sym_adj<<<grid_for(p, 128), 128, 0, s>>>(p, P.rp.p, P.ci.p, tptr.p, tlist.p, 0, acnt.p, nullptr, nullptr);
        VB_LAUNCH_CHECK();
    }
    const int64_t na = scan_i64(acnt.p, aptr.p, p, s);
    DBuf<int> adj(std::max<int64_t>(na, 1));
    if (p > 0) {
        k_sym_adj<<<grid_for(p, 128), 128, 0, s>>>(p, P.rp.p, P.ci.p, tptr.p, tlist.p, 1, nullptr, aptr.p, adj.p);
        VB_LAUNCH_CHECK();
    }
    char *stage = (char *)pinned_staging(sizeof(int64_t) * (p + 1) + sizeof(int) * (na + 1));
    hap = (const int64_t *)stage;
    hadj = (const int *)(stage + sizeof(int64_t) * (p + 1));
    VB_HIP(hipMemcpyAsync((void *)hap, aptr.p, sizeof(int64_t) * (p + 1), hipMemcpyDeviceToHost, s));
    if (na) VB_HIP(hipMemcpyAsync((void *)hadj, adj.p, sizeof(int) * na, hipMemcpyDeviceToHost, s));
    VB_HIP(hipEventRecord(ready, s));
}

// Upper bound of the distinct coarse block columns of every coarse block row.
__global__ void k_rg_bound(int pc, const int *mptr, const int *mem, const int64_t *rp, int64_t *cnt) {
    int X = blockIdx.x * blockDim.x + threadIdx.x;
    if (X >= pc) return;
    int64_t c = 0;
    for (int a = mptr[X]; a < mptr[X + 1]; ++a) c += rp[mem[a] + 1] - rp[mem[a]];
    cnt[X] = c;
}
// Coarse block columns of every coarse row: the members' block columns mapped to their
// coarse blocks, sorted and deduplicated in place; cnt[X] = distinct count.
__global__ void k_rg_cand(int pc, const int *mptr, const int *mem, const int64_t *rp, const int *ci, const int *cblk,
                          const int64_t *off, int *cand, int64_t *cnt) {
    int X = blockIdx.x * blockDim.x + threadIdx.x;
    if (X >= pc) return;
    int *c = cand + off[X];
    int64_t k2 = 0;
    for (int a = mptr[X]; a < mptr[X + 1]; ++a) {
        const int I = mem[a];
        for (int64_t k = rp[I]; k < rp[I + 1]; ++k) c[k2++] = cblk[ci[k]];
    }
    dev_shell_sort(c, k2);  // several hundred entries for a group of many members
    int64_t u = 0;
    for (int64_t i = 0; i < k2; ++i)
        if (u == 0 || c[i] != c[u - 1]) c[u++] = c[i];
    cnt[X] = u;
}
__global__ void k_rg_cols(int pc, const int64_t *off, const int *cand, const int64_t *crp, int *cci) {
    int X = blockIdx.x * blockDim.x + threadIdx.x;
    if (X >= pc) return;
    for (int64_t k = crp[X]; k < crp[X + 1]; ++k) cci[k] = cand[off[X] + (k - crp[X])];
}
// level row of every coarse row: crow[coarse row] = level row
__global__ void k_rg_crow(int p, const int *rb, const int *cblk, const int *coff, const int *crb, int *crow) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    const int base = crb[cblk[I]] + coff[I];
    for (int r = 0; r < rb[I + 1] - rb[I]; ++r) crow[base + r] = rb[I] + r;
}
// Coarse panel column of every panel column of the level matrix: block (I, J) lands in
// coarse block (cblk[I], cblk[J]) at column offset coff[J].  One thread per block.
__global__ void k_rg_cols_map(int p, int64_t nb, const int *rb, const int64_t *rp, const int *ci, const int *co,
                              const int64_t *wp, const int *cblk, const int *coff, const int64_t *crp, const int *cci,
                              const int *cco, int *dstpc, int *err) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const int I = (int)dev_floor(rp, 0, p + 1, k);
    const int X = cblk[I];
    const int J = ci[k];
    const int64_t pos = dev_find(cci, crp[X], crp[X + 1], cblk[J]);
    if (pos < 0) { dev_set_error(err, VBARMS_ERR_HIP, 2010, I); return; }
    const int dc = cco[pos] + coff[J];
    int *d = dstpc + wp[I] + co[k];
    for (int c = 0; c < rb[J + 1] - rb[J]; ++c) d[c] = dc + c;
}
// Scatter of the level matrix into the coarse panel (zeroed beforehand): 16 lanes per level
// row stream its panel row; row r of block I is row coff[I] + r of coarse block cblk[I].
template <class T>
__global__ void k_rg_vals(int n, const int *rowblk, const int *rb, const int64_t *wp, const int64_t *vp, const T *v,
                          const int *cblk, const int *coff, const int *dstpc, const int64_t *cwp, const int64_t *cvp,
                          T *cv) {
    constexpr int G = 16;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t fr = gid / G;
    const int lane = (int)(gid % G);
    if (fr >= n) return;
    const int I = rowblk[fr];
    const int r = (int)(fr - rb[I]);
    const int X = cblk[I];
    const int64_t W = wp[I + 1] - wp[I], CW = cwp[X + 1] - cwp[X];
    const T *src = v + vp[I] + r * W;
    T *dst = cv + cvp[X] + (int64_t)(coff[I] + r) * CW;
    const int *pc = dstpc + wp[I];
    for (int64_t c = lane; c < W; c += G) dst[pc[c]] = src[c];
}
// level row of every row of a block list, in the list's own numbering (IS or rest)
__global__ void k_row_maps(int nb, const int *list, const int *rb, const int *off, const int *crow, int *out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int I = list[i];
    for (int r = 0; r < rb[I + 1] - rb[I]; ++r) out[off[i] + r] = crow ? crow[rb[I] + r] : rb[I] + r;
}

// The level matrix with every group merged into one block: coarse blocks 0 .. ng-1 are
// the groups, then the remaining supernodes ascending.  crow receives the level row of
// every coarse row.
template <class T>
void regroup_panel(const Panel<T> &A, const HostGroups &G, Panel<T> &Ac, DBuf<int> &crow, int *err, hipStream_t s) {
    const int p = A.p;
    const int n = A.h_rb.back();
    std::vector<int> cblk(p), coff(p), mptr(1, 0), mem;
    std::vector<int> crb(1, 0);
    mem.reserve(p);
    for (int g = 0; g < G.ng; ++g) {
        int rows = 0;
        for (int a = G.gptr[g]; a < G.gptr[g + 1]; ++a) {
            const int I = G.members[a];
            cblk[I] = g;
            coff[I] = rows;
            rows += A.h_rb[I + 1] - A.h_rb[I];
            mem.push_back(I);
        }
        mptr.push_back((int)mem.size());
        crb.push_back(crb.back() + rows);
    }
    int X = G.ng;
    for (int I = 0; I < p; ++I) {
        if (G.gid[I] >= 0) continue;
        cblk[I] = X++;
        coff[I] = 0;
        mem.push_back(I);
        mptr.push_back((int)mem.size());
        crb.push_back(crb.back() + A.h_rb[I + 1] - A.h_rb[I]);
    }
    const int pc = X;
    DBuf<int> d_cblk(std::max(p, 1)), d_coff(std::max(p, 1)), d_mptr(pc + 1), d_mem(std::max(p, 1));
    to_device(d_cblk.p, cblk.data(), p, s);
    to_device(d_coff.p, coff.data(), p, s);
    to_device(d_mptr.p, mptr.data(), pc + 1, s);
    to_device(d_mem.p, mem.data(), p, s);
    panel_set_blocks(Ac, crb, crb, s);
    Ac.rp.alloc(pc + 1);
    {
        DBuf<int64_t> bound(std::max(pc, 1)), off(pc + 1), cnt(std::max(pc, 1));
        if (pc > 0) {
            k_rg_bound<<<grid_for(pc, 256), 256, 0, s>>>(pc, d_mptr.p, d_mem.p, A.rp.p, bound.p);
            VB_LAUNCH_CHECK();
        }
        const int64_t tot = scan_i64(bound.p, off.p, pc, s);
        DBuf<int> cand(std::max<int64_t>(tot, 1));
        if (pc > 0) {
            k_rg_cand<<<grid_for(pc, 64), 64, 0, s>>>(pc, d_mptr.p, d_mem.p, A.rp.p, A.ci.p, d_cblk.p, off.p, cand.p,
                                                       cnt.p);
            VB_LAUNCH_CHECK();
        }
        Ac.nb = scan_i64(cnt.p, Ac.rp.p, pc, s);
        Ac.ci.alloc(std::max<int64_t>(Ac.nb, 1));
        if (pc > 0) {
            k_rg_cols<<<grid_for(pc, 256), 256, 0, s>>>(pc, off.p, cand.p, Ac.rp.p, Ac.ci.p);
            VB_LAUNCH_CHECK();
        }
        VB_HIP(hipStreamSynchronize(s));  // host vectors above are copy sources
    }
    panel_finish_layout(Ac, s);
    Ac.v.alloc(std::max<int64_t>(Ac.nv, 1));
    fill_val<T>(Ac.v.p, T(0), Ac.nv, s);
    crow.alloc(std::max(n, 1));
    if (p > 0) {
        k_rg_crow<<<grid_for(p, 256), 256, 0, s>>>(p, A.rb.p, d_cblk.p, d_coff.p, Ac.rb.p, crow.p);
        VB_LAUNCH_CHECK();
    }
    if (p > 0) {
        DBuf<int> dstpc(std::max<int64_t>(A.nw, 1));
        if (A.nb > 0) {
            k_rg_cols_map<<<grid_for(A.nb, 256), 256, 0, s>>>(p, A.nb, A.rb.p, A.rp.p, A.ci.p, A.co.p, A.wp.p, d_cblk.p,
                                                               d_coff.p, Ac.rp.p, Ac.ci.p, Ac.co.p, dstpc.p, err);
            VB_LAUNCH_CHECK();
        }
        k_rg_vals<T><<<grid_for((int64_t)n * 16, 256), 256, 0, s>>>(n, A.rowblk.p, A.rb.p, A.wp.p, A.vp.p, A.v.p,
                                                                     d_cblk.p, d_coff.p, dstpc.p, Ac.wp.p, Ac.vp.p,
                                                                     Ac.v.p);
        VB_LAUNCH_CHECK();
    }
}

}  // namespace

template <class T>
void factor_level(Level<T> &L, Panel<T> &&Ain, int lvl, double droptol, int drop_schur, int is_order,
                  int group_rows, double min_ratio, Panel<T> &next, int *err, hipStream_t s) {
    L.A = std::move(Ain);
    const Panel<T> &A = L.A;
    L.p = A.p;
    L.n = A.h_rb.empty() ? 0 : A.h_rb.back();
    const int p = L.p, n = L.n;
    if (A.maxm > VBARMS_MAX_BLOCK) fail(VBARMS_ERR_OOM, "block larger than VBARMS_MAX_BLOCK");

    // Step 3 with groups in natural order needs only the pattern: its neighbour lists go to
    // the host first, so that the host greedy below runs while the device scales
    const bool grouped = group_rows > 0;
    const bool early_adjacency = grouped && is_order != 1;
    const int64_t *hap = nullptr;
    const int *hadj = nullptr;
    struct Event {
        hipEvent_t e = nullptr;
        ~Event() {
            if (e) (void)hipEventDestroy(e);
        }
    } adj_ready;
    if (grouped) VB_HIP(hipEventCreateWithFlags(&adj_ready.e, hipEventDisableTiming));
    if (early_adjacency) sym_adjacency_to_host(L.A, s, adj_ready.e, hap, hadj);

    // Step 2: scaling
    L.s1.alloc(std::max(n, 1));
    L.s2.alloc(std::max(n, 1));
    {
        DBuf<unsigned long long> cm(std::max(n, 1));
        fill_val<unsigned long long>(cm.p, 0ull, n, s);
        unsigned g = grid_for((int64_t)n * kTG, 256);
        k_rowmax<T><<<g, 256, 0, s>>>(n, A.rowblk.p, A.rb.p, A.wp.p, A.vp.p, A.v.p, L.s1.p);
        VB_LAUNCH_CHECK();
        if (p > 0) {
            k_colmax<T><<<grid_for((int64_t)p * kTG, 256), 256, 0, s>>>(p, A.rb.p, A.wp.p, A.vp.p, A.sc.p, A.v.p,
                                                                       L.s1.p, cm.p);
            VB_LAUNCH_CHECK();
        }
        k_s2<<<grid_for(n, 256), 256, 0, s>>>(n, cm.p, L.s2.p);
        VB_LAUNCH_CHECK();
        // scaled copy shares the layout
        panel_convert<T, T>(A, L.As, s);
        k_scale<T><<<g, 256, 0, s>>>(n, A.rowblk.p, A.rb.p, A.wp.p, A.vp.p, A.sc.p, A.v.p, L.s1.p, L.s2.p, L.As.v.p);
        VB_LAUNCH_CHECK();
    }
    // Step 3: block independent set on the quotient graph of A + A^T, in natural order or
    // by descending weight; either one supernode per group (parallel LFMIS rounds) or
    // groups of several supernodes merged into one block of a coarse copy of the matrix
    Panel<T> Ac;       // grouped: the level matrix with every group as one block
    DBuf<int> crow;    // grouped: level row of every row of Ac
    HostGroups G;
    DBuf<int> state;
    {
        const Panel<T> &As = L.As;
        DBuf<double> wts;
        if (is_order == 1 && p > 0) {
            wts.alloc(p);
            k_is_weights<T><<<grid_for(p, 256), 256, 0, s>>>(p, As.rb.p, As.rp.p, As.ci.p, As.co.p, As.wp.p, As.vp.p,
                                                             As.v.p, wts.p);
            VB_LAUNCH_CHECK();
        }
        if (grouped) {
            std::vector<double> hw;
            if (!early_adjacency) sym_adjacency_to_host(As, s, adj_ready.e, hap, hadj);
            VB_HIP(hipEventSynchronize(adj_ready.e));
            if (is_order == 1) to_host(hw, wts.p, p, s);
            G = host_groups(p, hap, hadj, As.h_rb, group_rows, is_order == 1 ? &hw : nullptr);
            regroup_panel(As, G, Ac, crow, err, s);
            state.alloc(std::max(Ac.p, 1));
            fill_i32(state.p, 1, G.ng, s);
            fill_i32(state.p + G.ng, 2, Ac.p - G.ng, s);
            L.h_members = G.members;
            L.h_gptr = G.gptr;
        } else {
            state.alloc(std::max(p, 1));
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
            L.h_members.clear();
            L.h_gptr.clear();
        }
    }
    // from here on the working matrix: the scaled level matrix, or its grouped copy
    const Panel<T> &As = grouped ? Ac : L.As;
    const int pw = As.p;

    // P_I: independent blocks ascending, then the rest ascending
    L.is_flag.alloc(std::max(pw, 1));
    L.num.alloc(std::max(pw, 1));
    {
        DBuf<int> restf(std::max(pw, 1)), issz(std::max(pw, 1)), restsz(std::max(pw, 1));
        DBuf<int> isidx(pw + 1), restidx(pw + 1), isoff(pw + 1), restoff(pw + 1);
        if (pw > 0) {
            k_is_flags<<<grid_for(pw, 256), 256, 0, s>>>(pw, state.p, As.rb.p, L.is_flag.p, restf.p, issz.p, restsz.p);
            VB_LAUNCH_CHECK();
        }
        L.nis = scan_i32(L.is_flag.p, isidx.p, pw, s);
        L.nrest = pw - L.nis;
        scan_i32(restf.p, restidx.p, pw, s, false);
        L.n_is = scan_i32(issz.p, isoff.p, pw, s);
        L.n_rest = n - L.n_is;
        scan_i32(restsz.p, restoff.p, pw, s, false);
        L.is_list.alloc(std::max(L.nis, 1));
        L.rest_list.alloc(std::max(L.nrest, 1));
        L.is_rb.alloc(L.nis + 1);
        L.rest_rb.alloc(L.nrest + 1);
        if (pw > 0) {
            k_numbering<<<grid_for(pw, 256), 256, 0, s>>>(pw, L.is_flag.p, isidx.p, restidx.p, isoff.p, restoff.p,
                                                          L.num.p, L.is_list.p, L.rest_list.p, L.is_rb.p, L.rest_rb.p);
            VB_LAUNCH_CHECK();
        }
        VB_HIP(hipMemcpyAsync(L.is_rb.p + L.nis, &L.n_is, sizeof(int), hipMemcpyHostToDevice, s));
        VB_HIP(hipMemcpyAsync(L.rest_rb.p + L.nrest, &L.n_rest, sizeof(int), hipMemcpyHostToDevice, s));
        to_host(L.h_is_rb, L.is_rb.p, L.nis + 1, s);
        to_host(L.h_rest_rb, L.rest_rb.p, L.nrest + 1, s);
    }
    L.nis_sn = grouped ? (int)G.members.size() : L.nis;
    L.is_rows.alloc(std::max(L.n_is, 1));
    L.rest_rows.alloc(std::max(L.n_rest, 1));
    if (L.nis > 0) {
        k_row_maps<<<grid_for(L.nis, 256), 256, 0, s>>>(L.nis, L.is_list.p, As.rb.p, L.is_rb.p,
                                                         grouped ? crow.p : nullptr, L.is_rows.p);
        VB_LAUNCH_CHECK();
    }
    if (L.nrest > 0) {
        k_row_maps<<<grid_for(L.nrest, 256), 256, 0, s>>>(L.nrest, L.rest_list.p, As.rb.p, L.rest_rb.p,
                                                           grouped ? crow.p : nullptr, L.rest_rows.p);
        VB_LAUNCH_CHECK();
    }
    const int nis = L.nis, nrest = L.nrest;

    // Step 4: pivot blocks
    L.dperm.alloc(std::max(L.n_is, 1));  // row exchanges of every pivot block as a permutation
    const DBuf<int> &dperm = L.dperm;
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
            k_gepp<T><<<grid_for(nis, 4), 256, 0, s>>>(nis, L.is_list.p, As.rb.p, As.rp.p, As.ci.p, As.co.p, As.wp.p,
                                                      As.vp.p, As.v.p, L.dlu_off.p, L.is_rb.p, L.dlu.p, L.dpiv.p, dperm.p,
                                                      min_ratio, lvl,
                                                      err);
            VB_LAUNCH_CHECK();
        }
        if (read_one(err, s) != 0) {
            if (grouped) {  // report the group's smallest supernode, as in the level numbering
                int rec[3];
                VB_HIP(hipMemcpyAsync(rec, err, sizeof(rec), hipMemcpyDeviceToHost, s));
                VB_HIP(hipStreamSynchronize(s));
                if (rec[0] == VBARMS_ERR_SINGULAR && rec[2] >= 0 && rec[2] < G.ng) {
                    rec[2] = G.members[G.gptr[rec[2]]];
                    VB_HIP(hipMemcpyAsync(err + 2, rec + 2, sizeof(int), hipMemcpyHostToDevice, s));
                    VB_HIP(hipStreamSynchronize(s));
                }
            }
            return;
        }
    }

    // G = L^{-1} P F and W = E U^{-1} into one scratch copy (their blocks are disjoint)
    DBuf<T> tmp(std::max<int64_t>(As.nv, 1));
    DBuf<int> keep(std::max<int64_t>(As.nb, 1));
    if (As.nw > 0) {
        k_compute_g<T><<<grid_for(As.nw, 128), 128, 0, s>>>(pw, As.nw, As.wp.p, As.vp.p, As.rb.p, As.sc.p,
                                                             As.rowblk.p, L.is_flag.p, L.num.p, As.v.p, L.dlu.p,
                                                             L.dlu_off.p, dperm.p, L.is_rb.p, tmp.p);
        VB_LAUNCH_CHECK();
        k_compute_w<T><<<grid_for(n, 128), 128, 0, s>>>(n, As.rowblk.p, As.rp.p, As.ci.p, As.co.p,
                                                                       As.wp.p, As.vp.p, As.rb.p, L.is_flag.p,
                                                                       L.num.p, As.v.p, L.dlu.p, L.dlu_off.p, tmp.p);
        VB_LAUNCH_CHECK();
    }
    if (As.nb > 0) {
        k_keep_gw<T><<<grid_for(As.nb, 256), 256, 0, s>>>(pw, As.nb, As.rp.p, As.ci.p, As.co.p, As.wp.p, As.vp.p,
                                                           As.rb.p, L.is_flag.p, tmp.p, droptol, 0, keep.p);
        VB_LAUNCH_CHECK();
    }
    panel_compact<T>(As, tmp.p, keep.p, L.is_list.p, nis, L.num.p, L.h_is_rb, L.h_rest_rb, L.G, s);
    if (As.nb > 0) {
        k_keep_gw<T><<<grid_for(As.nb, 256), 256, 0, s>>>(pw, As.nb, As.rp.p, As.ci.p, As.co.p, As.wp.p, As.vp.p,
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
    L.ws_nv = 0;  // apply workspaces are sized by the first application
}

template void factor_level<double>(Level<double> &, Panel<double> &&, int, double, int, int, int, double,
                                   Panel<double> &, int *, hipStream_t);
template void factor_level<float>(Level<float> &, Panel<float> &&, int, double, int, int, int, double, Panel<float> &,
                                  int *, hipStream_t);

}  // namespace vb
