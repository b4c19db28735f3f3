// Last-level block ILUT (Sec. 3, Alg. 3, IKJ order) and its block triangular solves.
//
// Factorization in dependency waves.  Every block row keeps its working row (block list,
// per-block state and dense blocks) in HBM.  One launch processes the ready rows: a row
// eliminates, in ascending column order exactly like the sequential IKJ loop, every block
// left of its diagonal whose row was finished in an EARLIER launch; when the next block to
// eliminate belongs to a row that is not finished yet, the row stops and waits for that
// row and its next few pending columns, and resumes in a later launch.  Data of other rows is only read across a kernel boundary,
// so no wait, flag protocol or fence is needed inside a kernel.  The smallest unfinished
// row can never stop, so every launch finishes at least one row.  Finished rows append
// their L and U blocks to pools, compacted into panels at the end.
//
// Solves: level scheduling from the final patterns of L and U; one launch per level, one
// wavefront per block row of the level.
#include <algorithm>
#include <climits>

#include "factor.h"

namespace vb {

namespace {

// launch shape of the wave kernel (a build may override the defaults for tuning sweeps)
#ifndef VB_ILUT_THREADS
#define VB_ILUT_THREADS 256
#endif
#ifndef VB_ILUT_GRID
#define VB_ILUT_GRID 1024
#endif
#ifndef VB_ILUT_USTAGE
#define VB_ILUT_USTAGE 1024
#endif
#ifndef VB_ILUT_STEPCAP
#define VB_ILUT_STEPCAP 8
#endif
// at least four resident wavefronts per SIMD (at most 128 registers per lane), so that the
// 1024 workgroups of a launch are resident together
#ifndef VB_ILUT_MINWAVES
#define VB_ILUT_MINWAVES 4
#endif
constexpr int kIlutThreads = VB_ILUT_THREADS;
static_assert(kIlutThreads % 64 == 0, "whole wavefronts");
constexpr int kMaxRowBlocks = 1024;  // largest block list of one working row
constexpr int kUStage = VB_ILUT_USTAGE;  // values of one LDS tile of U row k
constexpr int kCheckEvery = 16;      // ILUT waves between host checks
constexpr int kStepCap = VB_ILUT_STEPCAP;  // elimination steps a row takes per launch (the
                                           // smallest ready row is exempt)
constexpr int kIlutGrid = VB_ILUT_GRID;    // workgroups of every ILUT launch
constexpr int kGatherBlocks = 256;   // workgroups of the gather kernel

// sizes of the dynamic LDS of the ILUT wave kernel
struct IlutLds {
    int maxm;    // largest block size
    int rbcap;   // largest block list of a working row
    int hcap;    // hash capacity (power of two >= 1.5 rbcap)
    int ustage;  // values of one tile of U row k
};
template <class T>
size_t ilut_lds_bytes(const IlutLds &l) {
    size_t b = sizeof(T) * ((size_t)2 * l.maxm * l.maxm + l.ustage) +
               sizeof(int) * ((size_t)2 * l.hcap + 6 * l.rbcap + l.maxm + l.ustage) + (size_t)l.rbcap;
    return (b + 15) & ~(size_t)15;
}

struct IlutRowRec {
    int64_t lb, lv, ub, uv;  // block / value offsets in the pools
    int lc, lw, uc, uw;      // block counts and panel widths
    int64_t lu0;             // offset of the pivot-block LU factors
    int rbeg, m;             // first scalar row and size of the block row
};
struct RowState {
    int nb, used, last_k, status;  // status: 0 not started, 1 started, 2 finished
};
// Waiting-list entry: a row and the rows it awaits (-1: none).  A row that stops at an
// unfinished row k awaits k and its next pending columns, up to kWaitCols in ascending
// order, so that it runs again only once it can take that many steps; a row that stopped
// at the step cap awaits k alone.  Longer lists cut the visits further but defer rows
// until their backlog exceeds the step cap, which lengthens the chain of launches: of 1,
// 3, 7 and 15 columns, 3 took the least time on a 74^3-node upwind matrix.
#ifndef VB_ILUT_WAITCOLS
#define VB_ILUT_WAITCOLS 3
#endif
constexpr int kWaitCols = VB_ILUT_WAITCOLS;
struct __align__(16) IlutWait {
    int row;
    int k[kWaitCols];
};
static_assert(sizeof(IlutWait) % 16 == 0, "whole 16-byte words");
static_assert(kWaitCols >= 2, "k and at least one more column");
// a <- the N smallest of the ascending list a and the list b, whose columns are distinct
// from a's (INT_MAX: none); insertion with fixed indices, so both stay in registers
template <int N>
__device__ inline void wait_merge(int *a, const int *b) {
#pragma unroll
    for (int qb = 0; qb < N; ++qb) {
        int x = b[qb];
#pragma unroll
        for (int q = 0; q < N; ++q)
            if (x < a[q]) {
                const int tmp = a[q];
                a[q] = x;
                x = tmp;
            }
    }
}

// open-addressing hash in LDS (capacity hmask + 1, a power of two, at least 1.5 times the
// number of keys, so a probe always ends at a free slot)
__device__ inline int h_find(const int *keys, const int *vals, unsigned hmask, int key) {
    unsigned h = ((unsigned)key * 2654435761u) & hmask;
    for (;;) {
        int k = keys[h];
        if (k == key) return vals[h];
        if (k == -1) return -1;
        h = (h + 1) & hmask;
    }
}
__device__ inline void h_insert(int *keys, int *vals, unsigned hmask, int key, int val) {
    unsigned h = ((unsigned)key * 2654435761u) & hmask;
    for (;;) {
        int old = atomicCAS(&keys[h], -1, key);
        if (old == -1 || old == key) { vals[h] = val; return; }
        h = (h + 1) & hmask;
    }
}

// Multiplier solve x <- x U^{-1} L^{-1} P for a row x in registers and a pivot block of
// size MK held in LDS: the same operations in the same order as the generic row solves,
// so that only the (independent) loads of the LU factors remain in LDS.
template <class T, int MK>
__device__ inline void mult_solve_reg(const T *lu, const int *piv, T *x) {
#pragma unroll
    for (int c = 0; c < MK; ++c) {
        T s = x[c];
#pragma unroll
        for (int q = 0; q < c; ++q) s = s - x[q] * lu[q * MK + c];
        x[c] = s / lu[c * MK + c];
        // above 5 x 5, one column's LU loads at a time (bounds the registers in flight)
        if (MK > 5) __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int c = MK - 1; c >= 0; --c) {
        T s = x[c];
#pragma unroll
        for (int q = c + 1; q < MK; ++q) s = s - x[q] * lu[q * MK + c];
        x[c] = s;
        if (MK > 5) __builtin_amdgcn_sched_barrier(0);
    }
    // row interchanges, last pivot first, as selects over the register array
#pragma unroll
    for (int k = MK - 1; k >= 0; --k) {
        const int pk = piv[k];
        const T xk = x[k];
        T xp = xk;
#pragma unroll
        for (int j = 0; j < MK; ++j) xp = j == pk ? x[j] : xp;
#pragma unroll
        for (int j = 0; j < MK; ++j) x[j] = j == pk ? xk : x[j];
        x[k] = xp;
    }
}
// drop rule ||B||_F / (m n) < t for a contiguous row-major block: the squares are summed in
// index order like the generic test, with the loads issued four at a time
template <class T>
__device__ inline bool drop_contig(int m, int n, const T *b, double t) {
    const int cnt = m * n;
    T s = T(0);
    int q = 0;
    for (; q + 4 <= cnt; q += 4) {
        const T v0 = b[q], v1 = b[q + 1], v2 = b[q + 2], v3 = b[q + 3];
        s = s + v0 * v0;
        s = s + v1 * v1;
        s = s + v2 * v2;
        s = s + v3 * v3;
    }
    for (; q < cnt; ++q) {
        const T v = b[q];
        s = s + v * v;
    }
    const T thr = T(t) * T(cnt);
    return s < thr * thr;
}

// The m x mk multiplier block M (row-major in LDS) <- M U^{-1} L^{-1} P, one lane of the
// calling wavefront per row, followed by the drop rule ||M||_F / (m mk) < t.  The squares
// are summed in index order, one row after the other: each lane continues the running sum
// of the previous row's lane from its registers.  Returns the drop decision to every lane.
// Larger pivot blocks are solved in LDS (unrolled register solves of those sizes would
// cost the kernel a resident wavefront per SIMD).
template <class T, int MK>
__device__ inline bool mult_solve_drop_reg(int m, const T *lu, const int *piv, T *M, double t) {
    const int lane = threadIdx.x & 63;
    T x[MK];
#pragma unroll
    for (int c = 0; c < MK; ++c) x[c] = T(0);
    if (lane < m) {
        T *e = M + lane * MK;
#pragma unroll
        for (int c = 0; c < MK; ++c) x[c] = e[c];
        mult_solve_reg<T, MK>(lu, piv, x);
#pragma unroll
        for (int c = 0; c < MK; ++c) e[c] = x[c];
    }
    T s = T(0);
    for (int r = 0; r < m; ++r) {
        if (lane == r)
#pragma unroll
            for (int c = 0; c < MK; ++c) s = s + x[c] * x[c];
        s = __shfl(s, r, 64);
    }
    const T thr = T(t) * T(m * MK);
    return s < thr * thr;
}
template <class T>
__device__ inline bool mult_solve_drop(int m, int mk, const T *lu, const int *piv, T *M, double t) {
    switch (mk) {
        case 1: return mult_solve_drop_reg<T, 1>(m, lu, piv, M, t);
        case 2: return mult_solve_drop_reg<T, 2>(m, lu, piv, M, t);
        case 3: return mult_solve_drop_reg<T, 3>(m, lu, piv, M, t);
        case 4: return mult_solve_drop_reg<T, 4>(m, lu, piv, M, t);
        case 5: return mult_solve_drop_reg<T, 5>(m, lu, piv, M, t);
        // in single precision 6 x 6 and 7 x 7 also fit the kernel's register budget
        case 6:
            if constexpr (sizeof(T) == 4) return mult_solve_drop_reg<T, 6>(m, lu, piv, M, t);
            break;
        case 7:
            if constexpr (sizeof(T) == 4) return mult_solve_drop_reg<T, 7>(m, lu, piv, M, t);
            break;
        default: break;
    }
    const int lane = threadIdx.x & 63;
    if (lane < m) {
        dev_row_solve_u<T>(mk, lu, M + lane * mk, 1);
        dev_row_solve_lp<T>(mk, lu, piv, M + lane * mk, 1);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    return drop_contig<T>(m, mk, M, t);
}
// In-place exclusive prefix sums of a[0..n) (LDS) by the whole workgroup; returns the total
// to every thread.  Each thread sums a contiguous run of entries, the run sums are scanned
// within each wavefront and across the wavefronts (part: one int per wavefront), and the
// runs are rewritten.  Begins and ends with a barrier.
__device__ inline int wg_scan_excl(int *a, int n, int *part) {
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int run = (n + kIlutThreads - 1) / kIlutThreads;
    const int b = t * run, e = b + run < n ? b + run : n;
    __syncthreads();
    int sum = 0;
    for (int q = b; q < e; ++q) sum += a[q];
    int inc = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) part[wv] = inc;
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kIlutThreads / 64; ++q) {
        base += q < wv ? part[q] : 0;
        total += part[q];
    }
    int acc = base + inc - sum;
    for (int q = b; q < e; ++q) {
        const int v = a[q];
        a[q] = acc;
        acc += v;
    }
    __syncthreads();
    return total;
}
// The entry of a flat list that holds position q: the last e in [0, n) with pre[e] <= q
// (pre ascending, pre[0] = 0 <= q; an entry with no values shares its start with the next,
// so the last such e is the one whose values contain q).
__device__ inline int flat_entry(const int *pre, int n, int q) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Copies a rows x tw tile (row stride ld in global memory) to LDS (row stride tw) with nt
// threads (t = 0..nt-1).  Each thread issues up to six loads before it stores any, so the
// loads are in flight together.
template <class T>
__device__ inline void stage_tile(T *dst, const T *src, int64_t ld, int rows, int tw, int t, int nt) {
    constexpr int kPer = 6;
    const int tot = rows * tw;
    for (int e0 = 0; e0 < tot; e0 += kPer * nt) {
        T v[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = e0 + u * nt + t;
            v[u] = T(0);
            if (e < tot) {
                const int q = e / tw, cc = e - q * tw;
                v[u] = src[(int64_t)q * ld + cc];
            }
        }
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = e0 + u * nt + t;
            if (e < tot) dst[e] = v[u];
        }
    }
}

// One dependency wave of the block ILUT: one workgroup per row of the input list.
//
// The row's block list (column, value offset, state) lives in LDS for the launch and in
// its global region between launches; the dense blocks stay in the global region.  The
// pivot-block LU of row k, the multiplier block and U row k are staged in LDS before the
// small dense solves, which keep the operation order of the sequential algorithm.  A row
// that meets an unfinished row k saves its list and appends itself to the output list.
//
// A row that meets an unfinished row k records k, with its next pending columns, and
// appends itself to the waiting list; the gather kernel of a later launch returns it to the
// ready list once all of them have finished.
template <class T>
__device__ void ilut_row(
    const int i, int launch, int min_ready, int p, IlutWait *wait_out, int *cnt_wait_out, int *nfinished,
    const int *rb, const int64_t *rp, const int *ci, const int *co, const int64_t *wp, const int64_t *vp, const T *av,
    double droptol, double min_ratio, int *done, RowState *rs, const int64_t *boff, const int64_t *voff, int *wcols,
    int *woffs, unsigned char *west, T *wvals, T *dl, const int64_t *dl_off, int *dl_piv, IlutRowRec *rec, int *lci,
    int *lco,
    T *lv, int *uci, int *uco, T *uv, int64_t *cursors, int64_t capb_pool, int64_t capv_pool, int *err, int lvl,
    unsigned long long *moved, IlutLds lds) {
    // dynamic LDS, carved as described by `lds` (sizes chosen on the host for this matrix)
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *s_lu = (T *)lds_raw;                         // [maxm * maxm] pivot-block LU of row k
    T *s_M = s_lu + lds.maxm * lds.maxm;            // [maxm * maxm] multiplier block / pivot block
    T *s_U = s_M + lds.maxm * lds.maxm;             // [ustage] one tile of U row k
    int *hkeys = (int *)(s_U + lds.ustage);         // [hcap]
    int *hvals = hkeys + lds.hcap;                  // [hcap]
    int *l_cols = hvals + lds.hcap;                 // [rbcap] block list of the row
    int *l_offs = l_cols + lds.rbcap;               // [rbcap]
    int *s_ucol = l_offs + lds.rbcap;               // [rbcap] U row k: block columns,
    int *s_uc0 = s_ucol + lds.rbcap;                //   first panel columns,
    int *s_uoff = s_uc0 + lds.rbcap;                //   offsets of the matching blocks of w,
    int *s_un = s_uoff + lds.rbcap;                 //   block widths
    int *s_piv = s_un + lds.rbcap;                  // [maxm]
    int *s_cmap = s_piv + lds.maxm;                 // [ustage] per column of U row k: w offset
                                                    //   of the column (<< 6) | block width
    unsigned char *l_est = (unsigned char *)(s_cmap + lds.ustage);  // [rbcap] 0 pending, 1 eliminated,
                                                                    // 2 dropped (3/4: kept L/U)
    const unsigned hmask = (unsigned)lds.hcap - 1u;
    const int kRowCap = lds.rbcap;
    __shared__ int s_nb, s_used, s_last, s_status, s_stop, s_nb0;
    __shared__ int s_wmin[kIlutThreads / 64];
    __shared__ int s_wk[kIlutThreads / 64][kWaitCols - 1];
    __shared__ int s_drop;
    __shared__ int s_lc, s_lw, s_uc, s_uw;
    __shared__ int64_t s_lb, s_lv, s_ub, s_uv;
    const int t = threadIdx.x;
    constexpr int S = (int)sizeof(T);
    // algorithmic bytes of the work this row does in this launch (thread 0 keeps the sum)
    unsigned long long nbytes = 0;
    const int m = rb[i + 1] - rb[i];
    const int64_t B0 = boff[i], CB = boff[i + 1] - boff[i];
    const int64_t V0 = voff[i], CV = voff[i + 1] - voff[i];
    int *cols = wcols + B0;
    int *offs = woffs + B0;
    unsigned char *est = west + B0;
    T *w = wvals + V0;
    // the column map packs a w offset with a "new block" bit and the block width (6 bits)
    const bool use_map = CV < ((int64_t)1 << 24);
    // the first kSpecEntries saved list entries are loaded together with the row state (a
    // row's list region holds at least 64 entries; on a first visit they are not used)
    constexpr int kSpecEntries = 64;
    static_assert(kSpecEntries <= kIlutThreads, "one speculative entry per thread");
    const bool spec = t < kSpecEntries && t < CB;
    int spec_c = 0, spec_o = 0;
    unsigned char spec_s = 0;
    if (spec) {
        spec_c = cols[t];
        spec_o = offs[t];
        spec_s = est[t];
    }
    if (t == 0) {
        RowState r = rs[i];
        s_nb = r.nb;
        s_used = r.used;
        s_last = r.last_k;
        s_status = r.status;
        s_stop = 0;
        if (r.status == 0) {
            int nA = (int)(rp[i + 1] - rp[i]);
            int64_t W = wp[i + 1] - wp[i];
            if (nA > CB || m > lds.maxm || (int64_t)m * W > CV) {
                dev_set_error(err, VBARMS_ERR_OOM, lvl, i);  // the row's own room
                s_stop = 1;
            } else if (nA > kRowCap) {
                dev_set_error(err, VBARMS_ERR_OOM, lvl, -2 - i);  // the LDS block list
                s_stop = 1;
            }
            s_nb = nA;
            s_used = (int)(m * W);
            s_last = -1;
            nbytes += 2ull * S * m * W + 8ull * nA;  // row of A in, working row out
        } else {
            nbytes += 9ull * r.nb;  // saved block list back in
        }
    }
    __syncthreads();
    if (s_stop) return;
    if (s_status == 0) {
        // first visit: row i of A, one list entry per block, blocks stored contiguously;
        // the first panel columns of its blocks also go to s_uc0 for the copy below
        const int64_t b0 = rp[i];
        for (int e = t; e < s_nb; e += kIlutThreads) {
            const int c0 = co[b0 + e];
            l_cols[e] = ci[b0 + e];
            l_offs[e] = m * c0;
            l_est[e] = 0;
            s_uc0[e] = c0;
        }
    } else {
        // resumed row: the saved list; the speculative entries first, then the rest, four
        // entries per thread loaded before any is stored
        if (spec && t < s_nb) {
            l_cols[t] = spec_c;
            l_offs[t] = spec_o;
            l_est[t] = spec_s;
        }
        for (int e0 = 0; e0 + kSpecEntries < s_nb; e0 += 4 * kIlutThreads) {
            int cv[4], ov[4];
            unsigned char sv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = kSpecEntries + e0 + u * kIlutThreads + t;
                cv[u] = ov[u] = 0;
                sv[u] = 0;
                if (e < s_nb) {
                    cv[u] = cols[e];
                    ov[u] = offs[e];
                    sv[u] = est[e];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = kSpecEntries + e0 + u * kIlutThreads + t;
                if (e < s_nb) {
                    l_cols[e] = cv[u];
                    l_offs[e] = ov[u];
                    l_est[e] = sv[u];
                }
            }
        }
    }
    for (int h = t; h < lds.hcap; h += kIlutThreads) hkeys[h] = -1;
    // entries below s_nb0 are already in the row's global list (not on a first visit)
    if (t == 0) s_nb0 = s_status == 0 ? 0 : s_nb;
    __syncthreads();
    if (s_status == 0) {
        // the dense blocks of row i of A go to w block by block (each block row-major);
        // the block of a panel column is found in LDS, and the m values of a column are
        // loaded (eight at a time) before they are stored
        const int nA = s_nb;
        const int64_t W = wp[i + 1] - wp[i];
        const T *A = av + vp[i];
        for (int64_t c = t; c < W; c += kIlutThreads) {
            const int b = (int)dev_floor32(s_uc0, 0, nA, (int)c);
            const int nJ = (b + 1 < nA ? s_uc0[b + 1] : (int)W) - s_uc0[b];
            const int local = (int)(c - s_uc0[b]);
            T *dst = w + m * s_uc0[b] + local;
            for (int r0 = 0; r0 < m; r0 += 8) {
                T v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = r0 + u < m ? A[(int64_t)(r0 + u) * W + c] : T(0);
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (r0 + u < m) dst[(r0 + u) * nJ] = v[u];
            }
        }
    }
    for (int e = t; e < s_nb; e += kIlutThreads) h_insert(hkeys, hvals, hmask, l_cols[e], e);
    __syncthreads();

    // the last eliminated column, kept by every thread (all threads take the same k)
    int last = s_last;
    for (int nstep = 0;; ++nstep) {
        {
            // next column to eliminate: the smallest pending column left of the diagonal;
            // one slot per wavefront, so no reset (and no barrier for it) is needed
            int mine = INT_MAX;
            for (int e = t; e < s_nb; e += kIlutThreads) {
                const int K = l_cols[e];
                if (K < i && K > last && l_est[e] == 0 && K < mine) mine = K;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const int o = __shfl_xor(mine, off, 64);
                mine = o < mine ? o : mine;
            }
            if ((t & 63) == 0) s_wmin[t >> 6] = mine;
        }
        __syncthreads();
        int k = s_wmin[0];
#pragma unroll
        for (int q = 1; q < kIlutThreads / 64; ++q) k = s_wmin[q] < k ? s_wmin[q] : k;
        if (k == INT_MAX) break;
        // Row k is usable only if an earlier launch finished it.  Every thread reads the flag
        // and the record itself: a row finished in an earlier launch is read the same by
        // all, and any other value (0, or this launch) means "not usable" to all, so the
        // decision is uniform without a broadcast.
        const int dk = done[k];
        const IlutRowRec rk = rec[k];
        const int ek = h_find(hkeys, hvals, hmask, k);
        // A row that has taken kStepCap steps in this launch stops here as if row k were
        // unfinished (the gather returns it to the ready list at once if k is finished): a
        // wave then lasts a bounded number of steps instead of the longest backlog of ready
        // eliminations.  The smallest ready row is exempt, so every launch still finishes it.
        const bool capped = nstep >= kStepCap && i != min_ready;
        if (capped || !(dk > 0 && dk < launch)) {
            // not usable now: save the state of the list (the columns and offsets of
            // entries loaded at the start of this visit are unchanged)
            {
                // the kWaitCols - 1 smallest pending columns after k (none at the step cap):
                // each thread keeps its smallest in ascending order, each wavefront merges
                // them, and thread 0 merges the wavefronts after the barrier
                int c[kWaitCols - 1];
#pragma unroll
                for (int q = 0; q < kWaitCols - 1; ++q) c[q] = INT_MAX;
                if (!capped)
                    for (int e = t; e < s_nb; e += kIlutThreads) {
                        int K = l_cols[e];
                        if (K <= k || K >= i || l_est[e] != 0) continue;
#pragma unroll
                        for (int q = 0; q < kWaitCols - 1; ++q)
                            if (K < c[q]) {
                                const int tmp = c[q];
                                c[q] = K;
                                K = tmp;
                            }
                    }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    int o[kWaitCols - 1];
#pragma unroll
                    for (int q = 0; q < kWaitCols - 1; ++q) o[q] = __shfl_xor(c[q], off, 64);
                    wait_merge<kWaitCols - 1>(c, o);
                }
                if ((t & 63) == 0)
#pragma unroll
                    for (int q = 0; q < kWaitCols - 1; ++q) s_wk[t >> 6][q] = c[q];
            }
            for (int e = t; e < s_nb; e += kIlutThreads) {
                if (e >= s_nb0) {
                    cols[e] = l_cols[e];
                    offs[e] = l_offs[e];
                }
                est[e] = l_est[e];
            }
            __syncthreads();
            if (t == 0) {
                int c[kWaitCols - 1];
#pragma unroll
                for (int q = 0; q < kWaitCols - 1; ++q) c[q] = s_wk[0][q];
                for (int w = 1; w < kIlutThreads / 64; ++w) {
                    int o[kWaitCols - 1];
#pragma unroll
                    for (int q = 0; q < kWaitCols - 1; ++q) o[q] = s_wk[w][q];
                    wait_merge<kWaitCols - 1>(c, o);
                }
                rs[i] = RowState{s_nb, s_used, last, 1};
                nbytes += 8ull * (s_nb - s_nb0) + s_nb + 16 + sizeof(IlutWait);
                // wait on row k (and the next pending ones); everything written here is read
                // in a later launch
                IlutWait wt;
                wt.row = i;
                wt.k[0] = k;
#pragma unroll
                for (int q = 0; q < kWaitCols - 1; ++q) wt.k[q + 1] = c[q] == INT_MAX ? -1 : c[q];
                wait_out[atomicAdd(cnt_wait_out, 1)] = wt;
                atomicAdd(moved, nbytes);
            }
            return;
        }
        const int mk = rk.m;
        const int UW = rk.uw;
        {
            // the finished row must describe ranges inside the pools
            const bool ok = ek >= 0 && ek < s_nb && rk.uc >= 0 && rk.uc <= kRowCap && rk.ub >= 0 &&
                            rk.ub + rk.uc <= capb_pool && UW >= 0 && rk.uv >= 0 &&
                            rk.uv + (int64_t)mk * UW <= capv_pool && mk >= 1 && mk <= lds.maxm &&
                            rk.rbeg == rb[k] && rk.lu0 >= 0;
            if (!ok) {
                if (t == 0) {
                    dev_set_error(err, VBARMS_ERR_HIP, lvl, i);
                    atomicAdd(moved, nbytes);
                }
                return;
            }
        }
        const int TW = lds.ustage / mk;
        // Wavefront 0 stages the pivot-block LU of row k, its pivots and the multiplier block,
        // and solves and tests the multiplier; meanwhile the other wavefronts stage U row k's
        // block lists and the first tile of its values.  One barrier joins them.
        constexpr int kUT = kIlutThreads > 64 ? 64 : 0;  // first thread that stages U row k
        if (t < 64) {
            const T *dkp = dl + rk.lu0;
            for (int e = t; e < mk * mk; e += 64) s_lu[e] = dkp[e];
            for (int q = t; q < mk; q += 64) s_piv[q] = dl_piv[rk.rbeg + q];
            const T *Mg = w + l_offs[ek];
            for (int e = t; e < m * mk; e += 64) s_M[e] = Mg[e];
        }
        if (t >= kUT) {
            for (int b = t - kUT; b < rk.uc; b += kIlutThreads - kUT) {
                s_ucol[b] = uci[rk.ub + b];
                s_uc0[b] = uco[rk.ub + b];
            }
            stage_tile<T>(s_U, uv + rk.uv, UW, mk, UW < TW ? UW : TW, t - kUT, kIlutThreads - kUT);
        }
        if (t < 64) {
            // the wavefront's own LDS stores are complete before its solve reads them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
            const bool d = mult_solve_drop<T>(m, mk, s_lu, s_piv, s_M, droptol);
            if (t == 0) s_drop = d ? 1 : 0;
        }
        __syncthreads();
        const bool dropped = s_drop != 0;
        if (t == 0) {
            // readiness and record of row k, its pivot block, the multiplier in and out
            nbytes += 68ull + (unsigned long long)S * mk * mk + 4ull * mk + 2ull * S * m * mk;
            // U row k with its block lists, and the read-modify-write of the updated blocks
            if (!dropped) nbytes += (unsigned long long)S * mk * UW + 8ull * rk.uc + 2ull * S * m * UW;
        }
        if (dropped) {
            // the scan skips column k (k <= last), so the state byte needs no barrier here
            if (t == 0) l_est[ek] = 2;
            last = k;
            continue;
        }
        {
            T *Mg = w + l_offs[ek];
            for (int e = t; e < m * mk; e += kIlutThreads) Mg[e] = s_M[e];
        }
        if (t == 0) l_est[ek] = 1;
        // fill: blocks of U row k not yet in the working row; every block of U row k
        // records where its counterpart lives in w
        for (int b = t; b < rk.uc; b += kIlutThreads) {
            const int J = s_ucol[b];
            const int nJ = (b + 1 < rk.uc ? s_uc0[b + 1] : UW) - s_uc0[b];
            if (J <= k || J >= p || nJ < 1 || nJ > lds.maxm) {
                dev_set_error(err, VBARMS_ERR_HIP, lvl, i);
                s_stop = 1;
                continue;
            }
            s_un[b] = nJ;
            const int e0 = h_find(hkeys, hvals, hmask, J);
            if (e0 >= 0) {
                const int off = l_offs[e0];
                s_uoff[b] = off;
                if (use_map)
                    for (int q = 0; q < nJ && s_uc0[b] + q < lds.ustage; ++q) s_cmap[s_uc0[b] + q] = ((off + q) << 7) | nJ;
                continue;
            }
            int e = atomicAdd(&s_nb, 1);
            int off = atomicAdd(&s_used, m * nJ);
            if (e >= CB || e >= kRowCap || (int64_t)off + m * nJ > CV) {
                // the row's own room (block >= 0) or the LDS block list (block <= -2) is full
                dev_set_error(err, VBARMS_ERR_OOM, lvl, e >= CB || (int64_t)off + m * nJ > CV ? i : -2 - i);
                s_stop = 1;
                continue;
            }
            l_cols[e] = J;
            l_offs[e] = off;
            l_est[e] = 0;
            s_uoff[b] = off;
            // a new block starts from zero: the update below writes every value of it
            // without reading w first, so it needs no clearing
            s_un[b] = nJ | 256;
            if (use_map)
                for (int q = 0; q < nJ && s_uc0[b] + q < lds.ustage; ++q)
                    s_cmap[s_uc0[b] + q] = ((off + q) << 7) | 64 | nJ;
            h_insert(hkeys, hvals, hmask, J, e);
        }
        // LDS only: the update reads the block list, the maps and the staged tiles from LDS;
        // the w blocks it reads were last written before the scan's full barrier, and the
        // multiplier block stored above is not read again in this step
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (s_stop) {
            if (t == 0) atomicAdd(moved, nbytes);
            return;
        }
        // w_J -= M U_kJ for every block J of U row k; U row k is staged in LDS one tile of
        // columns at a time (the first tile with the block lists) and the threads share the
        // (row, column) pairs of the tile
        for (int c0 = 0; c0 < UW; c0 += TW) {
            const int tw = UW - c0 < TW ? UW - c0 : TW;
            if (c0 > 0) {
                __syncthreads();  // the previous tile is consumed
                stage_tile<T>(s_U, uv + rk.uv + c0, UW, mk, tw, t, kIlutThreads);
                __syncthreads();
            }
            // each thread takes up to four (row, column) pairs at a time and loads their w
            // values before it stores any, so the loads are in flight together (the pairs
            // are distinct entries of w)
            const int tot = m * tw;
            for (int e0 = 0; e0 < tot; e0 += 4 * kIlutThreads) {
                T *wq[4];
                T val[4];
                int rq[4], cq[4];
                bool fresh[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * kIlutThreads + t;
                    wq[u] = nullptr;
                    val[u] = T(0);
                    rq[u] = cq[u] = 0;
                    fresh[u] = false;
                    if (e < tot) {
                        const int r = e / tw, cc = e - r * tw, c = c0 + cc;
                        int base, nJ;
                        if (use_map && c < lds.ustage) {
                            const int code = s_cmap[c];
                            base = code >> 7;
                            fresh[u] = (code & 64) != 0;
                            nJ = code & 63;
                        } else {
                            const int b = (int)dev_floor32(s_uc0, 0, rk.uc, c);
                            nJ = s_un[b] & 255;
                            fresh[u] = s_un[b] > 255;
                            base = s_uoff[b] + (c - s_uc0[b]);
                        }
                        wq[u] = w + base + r * nJ;
                        rq[u] = r;
                        cq[u] = cc;
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (wq[u] && !fresh[u]) val[u] = *wq[u];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (!wq[u]) continue;
                    T acc = val[u];
                    for (int q = 0; q < mk; ++q) acc = acc - s_M[rq[u] * mk + q] * s_U[q * tw + cq[u]];
                    *wq[u] = acc;
                }
            }
        }
        // the barrier after the next scan orders these updates before any later read of w
        // and before the staging buffers are overwritten
        last = k;
    }

    // finalize row i: pivot block, dropped upper blocks, output to the pools
    const int ei = h_find(hkeys, hvals, hmask, i);
    if (ei >= 0)
        for (int e = t; e < m * m; e += kIlutThreads) s_M[e] = w[l_offs[ei] + e];
    // per entry: block width, and the value count of the upper blocks (tested below)
    for (int e = t; e < s_nb; e += kIlutThreads) {
        const int K = l_cols[e];
        const int nK = rb[K + 1] - rb[K];
        s_un[e] = nK;
        s_uoff[e] = K > i ? m * nK : 0;
    }
    __syncthreads();
    if (t < 64) {
        // the pivot block, factored by wavefront 0
        const bool ok = ei >= 0 && wave_gepp<T>(m, s_M, s_piv, t);
        if (t == 0) {
            s_lc = s_lw = s_uc = s_uw = 0;
            if (!ok) {
                dev_set_error(err, VBARMS_ERR_SINGULAR, lvl, i);
                if (ei < 0)
                    for (int q = 0; q < m * m; ++q) s_M[q] = T(0);
                for (int q = 0; q < m; ++q) s_piv[q] = q;
            } else {
                dev_count_illcond<T>(m, s_M, min_ratio, err);
            }
        }
    }
    // offsets of the upper blocks in one flat list; when they fit, they are staged in LDS in
    // one round of loads and tested there
    const int tu = wg_scan_excl(s_uoff, s_nb, s_wmin);
    const bool ustaged = tu <= lds.ustage;
    if (ustaged) {
        for (int q0 = 0; q0 < tu; q0 += 4 * kIlutThreads) {
            T v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kIlutThreads + t;
                v[u] = T(0);
                if (q < tu) {
                    const int e = flat_entry(s_uoff, s_nb, q);
                    v[u] = w[l_offs[e] + (q - s_uoff[e])];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kIlutThreads + t;
                if (q < tu) s_U[q] = v[u];
            }
        }
    }
    {
        T *d = dl + dl_off[i];
        for (int e = t; e < m * m; e += kIlutThreads) d[e] = s_M[e];
        for (int q = t; q < m; q += kIlutThreads) dl_piv[rb[i] + q] = s_piv[q];
    }
    __syncthreads();
    for (int e = t; e < s_nb; e += kIlutThreads) {
        const int K = l_cols[e];
        if (K < i) l_est[e] = l_est[e] == 1 ? 3 : 0;
        else if (K > i)
            l_est[e] = drop_contig<T>(m, s_un[e], ustaged ? s_U + s_uoff[e] : w + l_offs[e], droptol) ? 0 : 4;
        else l_est[e] = 0;
    }
    __syncthreads();
    for (int e = t; e < s_nb; e += kIlutThreads) {
        const int nK = s_un[e];
        if (l_est[e] == 3) { atomicAdd(&s_lc, 1); atomicAdd(&s_lw, nK); }
        if (l_est[e] == 4) { atomicAdd(&s_uc, 1); atomicAdd(&s_uw, nK); }
    }
    __syncthreads();
    if (t == 0) {
        s_lb = (int64_t)atomicAdd((unsigned long long *)&cursors[0], (unsigned long long)s_lc);
        s_lv = (int64_t)atomicAdd((unsigned long long *)&cursors[1], (unsigned long long)m * s_lw);
        s_ub = (int64_t)atomicAdd((unsigned long long *)&cursors[2], (unsigned long long)s_uc);
        s_uv = (int64_t)atomicAdd((unsigned long long *)&cursors[3], (unsigned long long)m * s_uw);
        if (s_lb + s_lc > capb_pool || s_lv + (int64_t)m * s_lw > capv_pool || s_ub + s_uc > capb_pool ||
            s_uv + (int64_t)m * s_uw > capv_pool) {
            dev_set_error(err, VBARMS_ERR_OOM, lvl, -1);
            s_stop = 1;
        }
    }
    __syncthreads();
    if (s_stop) return;
    // output position = rank by block column; panel offset = widths of smaller columns; the
    // kept blocks' value counts give the flat list the copy below walks
    for (int e = t; e < s_nb; e += kIlutThreads) {
        const int st = l_est[e];
        int cnt = 0;
        if (st == 3 || st == 4) {
            const int K = l_cols[e];
            int rank = 0, off = 0;
            for (int f = 0; f < s_nb; ++f) {
                if (l_est[f] == st && l_cols[f] < K) {
                    ++rank;
                    off += s_un[f];
                }
            }
            if (st == 3) {
                lci[s_lb + rank] = K;
                lco[s_lb + rank] = off;
            } else {
                uci[s_ub + rank] = K;
                uco[s_ub + rank] = off;
            }
            s_ucol[e] = off;
            cnt = m * s_un[e];
        }
        s_uc0[e] = cnt;
    }
    const int tc = wg_scan_excl(s_uc0, s_nb, s_wmin);
    // the kept blocks' values to the panels, all threads over the flat list, four values
    // per thread loaded before any is stored
    for (int q0 = 0; q0 < tc; q0 += 4 * kIlutThreads) {
        T v[4];
        T *dst[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + u * kIlutThreads + t;
            v[u] = T(0);
            dst[u] = nullptr;
            if (q < tc) {
                const int e = flat_entry(s_uc0, s_nb, q);
                const int local = q - s_uc0[e], nK = s_un[e];
                const int r = local / nK, c = local - r * nK;
                if (l_est[e] == 3) {
                    dst[u] = lv + s_lv + (int64_t)r * s_lw + s_ucol[e] + c;
                    v[u] = w[l_offs[e] + local];
                } else {
                    dst[u] = uv + s_uv + (int64_t)r * s_uw + s_ucol[e] + c;
                    v[u] = ustaged ? s_U[s_uoff[e] + local] : w[l_offs[e] + local];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (dst[u]) *dst[u] = v[u];
    }
    if (t == 0) {
        rec[i] = IlutRowRec{s_lb, s_lv, s_ub, s_uv, s_lc, s_lw, s_uc, s_uw, dl_off[i], rb[i], m};
        rs[i] = RowState{s_nb, s_used, last, 2};
        done[i] = launch;
        atomicAdd(nfinished, 1);
        // pivot block in and its LU out, kept blocks copied to the pools, the records
        nbytes += 2ull * S * m * m + 4ull * m + 2ull * S * m * (s_lw + s_uw) + 8ull * (s_lc + s_uc) + 72;
        atomicAdd(moved, nbytes);
    }
}

// Gather of a launch: waiting rows whose awaited rows have all finished (in an earlier
// launch) move to the ready list, the others stay on the waiting list.  Rows that never ran
// await nothing.  Each workgroup takes 1024 consecutive entries at a time, four per thread
// with all loads issued before use, and appends them with one atomic per list (positions
// from wavefront ballots and an LDS scan over the wavefronts).
constexpr int kGatherThreads = 256;
constexpr int kGatherItems = 4;

__global__ void __launch_bounds__(kGatherThreads) k_ilut_gather(const IlutWait *wait_in, const int *cnt_wait_in,
                                                                const int *done, int *ready, int *cnt_ready,
                                                                IlutWait *wait_out, int *cnt_wait_out,
                                                                int *min_ready) {
    constexpr int NW = kGatherThreads / 64;
    __shared__ int s_tr[NW], s_tw[NW], s_br[NW], s_bw[NW], s_mn[NW];
    const int n = *cnt_wait_in;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const unsigned long long lt = (1ull << lane) - 1ull;
    constexpr int tile = kGatherThreads * kGatherItems;
    for (int b0 = blockIdx.x * tile; b0 < n; b0 += gridDim.x * tile) {
        IlutWait ent[kGatherItems];
        bool has[kGatherItems], rdy[kGatherItems];
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            const int e = b0 + u * kGatherThreads + t;
            has[u] = e < n;
            if (has[u]) {
                ent[u] = wait_in[e];
            } else {
                ent[u].row = -1;
#pragma unroll
                for (int q = 0; q < kWaitCols; ++q) ent[u].k[q] = -1;
            }
        }
        int dk[kGatherItems][kWaitCols];
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u)
#pragma unroll
            for (int q = 0; q < kWaitCols; ++q) dk[u][q] = ent[u].k[q] >= 0 ? done[ent[u].k[q]] : 1;
        int pr[kGatherItems], pw[kGatherItems];
        int tr = 0, tw = 0, mn = INT_MAX;
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            bool all = true;
#pragma unroll
            for (int q = 0; q < kWaitCols; ++q) all = all && dk[u][q] != 0;
            rdy[u] = has[u] && all;
            const unsigned long long mr = __ballot(rdy[u]), mw = __ballot(has[u] && !rdy[u]);
            pr[u] = tr + __popcll(mr & lt);
            pw[u] = tw + __popcll(mw & lt);
            tr += __popcll(mr);
            tw += __popcll(mw);
            if (rdy[u] && ent[u].row < mn) mn = ent[u].row;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const int o = __shfl_xor(mn, off, 64);
            mn = o < mn ? o : mn;
        }
        if (lane == 0) {
            s_tr[wv] = tr;
            s_tw[wv] = tw;
            s_mn[wv] = mn;
        }
        __syncthreads();
        if (t == 0) {
            int ar = 0, aw = 0, m = INT_MAX;
            for (int q = 0; q < NW; ++q) {
                s_br[q] = ar;
                s_bw[q] = aw;
                ar += s_tr[q];
                aw += s_tw[q];
                m = s_mn[q] < m ? s_mn[q] : m;
            }
            const int base_r = ar > 0 ? atomicAdd(cnt_ready, ar) : 0;
            const int base_w = aw > 0 ? atomicAdd(cnt_wait_out, aw) : 0;
            for (int q = 0; q < NW; ++q) {
                s_br[q] += base_r;
                s_bw[q] += base_w;
            }
            if (m != INT_MAX) atomicMin(min_ready, m);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kGatherItems; ++u) {
            if (!has[u]) continue;
            if (rdy[u]) ready[s_br[wv] + pr[u]] = ent[u].row;
            else wait_out[s_bw[wv] + pw[u]] = ent[u];
        }
        __syncthreads();  // s_br / s_bw are rewritten by the next tile
    }
}

// waiting list of the first launch: every row, awaiting nothing
__global__ void k_wait_init(int p, IlutWait *w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p) {
        IlutWait e;
        e.row = i;
#pragma unroll
        for (int q = 0; q < kWaitCols; ++q) e.k[q] = -1;
        w[i] = e;
    }
}

// One launch: a fixed grid strides over the ready list.  Counter slots: the gather of
// launch L fills the ready count and the waiting count this launch appends to; the wave
// clears the ready count of launch L+1 and the waiting count launch L+1 will append to,
// both last read by launch L-1.
template <class T>
__global__ void __launch_bounds__(kIlutThreads, VB_ILUT_MINWAVES) k_ilut_wave(
    int launch, int p, const int *ready, const int *cnt_ready, int *cnt_ready_clear, const int *min_ready_in,
    int *min_ready_clear, IlutWait *wait_out,
    int *cnt_wait_out, int *cnt_wait_clear, int *nfinished, const int *rb, const int64_t *rp,
    const int *ci, const int *co, const int64_t *wp, const int64_t *vp, const T *av, double droptol, double min_ratio,
    int *done, RowState *rs, const int64_t *boff, const int64_t *voff, int *wcols, int *woffs, unsigned char *west,
    T *wvals,
    T *dl, const int64_t *dl_off, int *dl_piv, IlutRowRec *rec, int *lci, int *lco, T *lv, int *uci, int *uco, T *uv,
    int64_t *cursors, int64_t capb_pool, int64_t capv_pool, int *err, int lvl, unsigned long long *moved,
    IlutLds lds) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *cnt_ready_clear = 0;
        *cnt_wait_clear = 0;
        *min_ready_clear = INT_MAX;
    }
    const int nin = *cnt_ready;
    const int min_ready = *min_ready_in;
    for (int slot = blockIdx.x; slot < nin; slot += gridDim.x) {
        ilut_row<T>(ready[slot], launch, min_ready, p, wait_out, cnt_wait_out, nfinished, rb, rp, ci, co, wp, vp, av,
                    droptol, min_ratio, done, rs, boff, voff, wcols, woffs, west, wvals, dl, dl_off, dl_piv, rec, lci,
                    lco, lv, uci,
                    uco, uv, cursors, capb_pool, capv_pool, err, lvl, moved, lds);
        __syncthreads();
    }
}

// capacities of the per-row working rows: `grow` times the input row, and at least `grow`
// times the mean input row (blocks, panel columns), so that short rows that fill up do not
// force a retry
__global__ void k_row_caps(int p, const int *rb, const int64_t *rp, const int64_t *wp, int grow, int64_t floor_b,
                           int64_t floor_w, int64_t *capb, int64_t *capv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    int64_t nA = rp[i + 1] - rp[i];
    int64_t m = rb[i + 1] - rb[i];
    int64_t W = wp[i + 1] - wp[i];
    capb[i] = std::min<int64_t>(kMaxRowBlocks, std::max<int64_t>(std::max<int64_t>(64, floor_b), grow * nA));
    capv[i] = m * std::max<int64_t>(std::max<int64_t>(64, floor_w), grow * W);
}

__global__ void k_rec_counts(int p, const IlutRowRec *rec, int which, int64_t *cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    cnt[i] = which == 0 ? rec[i].lc : rec[i].uc;
}
__global__ void k_pool_ci(int p, const IlutRowRec *rec, int which, const int *pci, const int64_t *rp, int *ci) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    int64_t b = which == 0 ? rec[i].lb : rec[i].ub;
    int c = which == 0 ? rec[i].lc : rec[i].uc;
    for (int k = 0; k < c; ++k) ci[rp[i] + k] = pci[b + k];
}
template <class T>
__global__ void k_pool_vals(int p, const int *rb, const IlutRowRec *rec, int which, const T *pv, const int64_t *vp,
                            T *v) {
    int i = blockIdx.x;
    int64_t src = which == 0 ? rec[i].lv : rec[i].uv;
    int w = which == 0 ? rec[i].lw : rec[i].uw;
    int64_t cnt = (int64_t)w * (rb[i + 1] - rb[i]);
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) v[vp[i] + e] = pv[src + e];
}

template <class T>
void pool_to_panel(int p, const std::vector<int> &rb, const DBuf<int> &drb, const IlutRowRec *rec, int which,
                   const int *pci, const T *pv, Panel<T> &out, hipStream_t s) {
    panel_set_blocks(out, rb, rb, s);
    out.rp.alloc(p + 1);
    DBuf<int64_t> cnt(std::max(p, 1));
    if (p > 0) {
        k_rec_counts<<<grid_for(p, 256), 256, 0, s>>>(p, rec, which, cnt.p);
        VB_LAUNCH_CHECK();
    }
    out.nb = scan_i64(cnt.p, out.rp.p, p, s);
    out.ci.alloc(std::max<int64_t>(out.nb, 1));
    if (p > 0) {
        k_pool_ci<<<grid_for(p, 256), 256, 0, s>>>(p, rec, which, pci, out.rp.p, out.ci.p);
        VB_LAUNCH_CHECK();
    }
    panel_finish_layout(out, s);
    out.v.alloc(std::max<int64_t>(out.nv, 1));
    if (p > 0) {
        k_pool_vals<T><<<p, 128, 0, s>>>(p, drb.p, rec, which, pv, out.vp.p, out.v.p);
        VB_LAUNCH_CHECK();
    }
}

__global__ void k_sq_sizes(int p, const int *rb, int64_t *sq) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p) sq[i] = (int64_t)(rb[i + 1] - rb[i]) * (rb[i + 1] - rb[i]);
}

// ---- level-scheduled block substitution ---------------------------------------------
constexpr int kSweepThreads = 256;

// Descriptor of one block row of a sweep, stored in level order so that a workgroup needs
// a single load to find its row.
struct SweepRow {
    int i, r_begin, m, pad;
    int64_t w0, W, v0, lu0;
};

// mode 0: t_i = b_i - sum_k L_ik t_k; mode 1: x_i = D_i^{-1}(t_i - sum_j U_ij x_j).
// One workgroup per block row of the current level (rows of a level are independent) and
// vector (blockIdx.y; b and x hold their vectors ld apart).
// The lanes of the workgroup are split evenly over the m scalar rows of the block row
// (a power-of-two group per row, at most 64 lanes), each group strides over the panel
// columns.  In mode 1 the pivot-block LU factors are staged in LDS and the small
// substitution runs on the first wavefront, one lane per scalar row.
template <class T>
__global__ void __launch_bounds__(kSweepThreads) k_trsv_level(const SweepRow *rows, int mode, const int *sc,
                                                              const T *v, const T *dl, const int *dl_piv,
                                                              const double *b, double *x, int64_t ld) {
    __shared__ double sv[VBARMS_MAX_BLOCK];
    b += blockIdx.y * ld;
    x += blockIdx.y * ld;
    __shared__ T slu[VBARMS_MAX_BLOCK * VBARMS_MAX_BLOCK];
    __shared__ int spiv[VBARMS_MAX_BLOCK];
    const int t = threadIdx.x;
    const SweepRow R = rows[blockIdx.x];
    const int m = R.m;
    if (mode == 1) {
        const T *d = dl + R.lu0;
        for (int e = t; e < m * m; e += kSweepThreads) slu[e] = d[e];
        if (t < m) spiv[t] = dl_piv[R.r_begin + t];
    }
    // lanes per scalar row: the largest power of two with m * tg <= threads, at most 64
    int tg = 64;
    while (tg > 1 && m * tg > kSweepThreads) tg >>= 1;
    const int grp = t / tg, gl = t % tg;
    const int *c = sc + R.w0;
    double acc = 0.0;
    if (grp < m) {
        // four columns per lane at a time: their indices, values and x entries are loaded
        // before any is used; the sum keeps the column order of the plain loop
        const T *a = v + R.v0 + (int64_t)grp * R.W;
        int64_t j = gl;
        for (; j + 3 * tg < R.W; j += 4 * tg) {
            const int c0 = c[j], c1 = c[j + tg], c2 = c[j + 2 * tg], c3 = c[j + 3 * tg];
            const T a0 = a[j], a1 = a[j + tg], a2 = a[j + 2 * tg], a3 = a[j + 3 * tg];
            const double x0 = x[c0], x1 = x[c1], x2 = x[c2], x3 = x[c3];
            acc += (double)a0 * x0;
            acc += (double)a1 * x1;
            acc += (double)a2 * x2;
            acc += (double)a3 * x3;
        }
        for (; j < R.W; j += tg) acc += (double)a[j] * x[c[j]];
    }
    for (int off = tg / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, tg);
    if (grp < m && gl == 0) sv[grp] = b[R.r_begin + grp] - acc;
    __syncthreads();
    if (mode == 1 && t < 64) {
        // x <- U^{-1} L^{-1} P y with one lane per scalar row (m <= 32)
        if (t == 0)
            for (int k = 0; k < m; ++k) {
                const int pk = spiv[k];
                if (pk != k) { double tmp = sv[k]; sv[k] = sv[pk]; sv[pk] = tmp; }
            }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        double y = t < m ? sv[t] : 0.0;
        for (int k = 0; k + 1 < m; ++k) {
            const double yk = __shfl(y, k, 64);
            if (t > k && t < m) y = y - (double)slu[t * m + k] * yk;
        }
        for (int k = m - 1; k >= 0; --k) {
            if (t == k) y = y / (double)slu[k * m + k];
            const double xk = __shfl(y, k, 64);
            if (t < k) y = y - (double)slu[t * m + k] * xk;
        }
        if (t < m) x[R.r_begin + t] = y;
    } else if (mode == 0 && t < m) {
        x[R.r_begin + t] = sv[t];
    }
}

// level schedule of a triangular block pattern; rows sorted by level, level offsets
void level_schedule(int p, const std::vector<int64_t> &rp, const std::vector<int> &ci,
                    bool descending, std::vector<int> &order, std::vector<int> &lptr) {
    std::vector<int> lev(p, 0);
    int maxl = -1;
    for (int s = 0; s < p; ++s) {
        int i = descending ? p - 1 - s : s;
        int l = 0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) l = std::max(l, lev[ci[k]] + 1);
        lev[i] = l;
        maxl = std::max(maxl, l);
    }
    lptr.assign(maxl + 2, 0);
    for (int i = 0; i < p; ++i) lptr[lev[i] + 1]++;
    for (int l = 0; l <= maxl; ++l) lptr[l + 1] += lptr[l];
    order.assign(p, 0);
    std::vector<int> fill(lptr.begin(), lptr.end() - 1);
    for (int s = 0; s < p; ++s) {
        int i = descending ? p - 1 - s : s;
        order[fill[lev[i]]++] = i;
    }
}

}  // namespace

template <class T>
void factor_last(LastLevel<T> &last, double droptol, double min_ratio, int lvl, IlutHint &hint, int *err,
                 hipStream_t s) {
    Panel<T> &A = last.A;
    const int p = A.p;
    const int n = A.h_rb.empty() ? 0 : A.h_rb.back();
    if (A.maxm > VBARMS_MAX_BLOCK) fail(VBARMS_ERR_OOM, "block larger than VBARMS_MAX_BLOCK");
    last.dl_off.alloc(p + 1);
    DBuf<int64_t> sq(std::max(p, 1));
    if (p > 0) {
        k_sq_sizes<<<grid_for(p, 256), 256, 0, s>>>(p, A.rb.p, sq.p);
        VB_LAUNCH_CHECK();
    }
    int64_t dtot = scan_i64(sq.p, last.dl_off.p, p, s);
    last.dl.alloc(std::max<int64_t>(dtot, 1));
    last.dl_piv.alloc(std::max(n, 1));
    last.t.alloc(std::max(n, 1));
    last.lorder.clear();
    last.uorder.clear();
    last.lptr.assign(1, 0);
    last.uptr.assign(1, 0);
    if (p == 0) {
        panel_set_blocks(last.L, A.h_rb, A.h_rb, s);
        panel_set_blocks(last.U, A.h_rb, A.h_rb, s);
        last.L.rp.alloc(1); fill_i64(last.L.rp.p, 0, 1, s); panel_finish_layout(last.L, s);
        last.U.rp.alloc(1); fill_i64(last.U.rp.p, 0, 1, s); panel_finish_layout(last.U, s);
        return;
    }
    int64_t max_na = 0;  // longest block row of the input
    {
        std::vector<int64_t> hrp;
        to_host(hrp, A.rp.p, p + 1, s);
        for (int i = 0; i < p; ++i) max_na = std::max(max_na, hrp[i + 1] - hrp[i]);
    }
    last.attempts = 0;
    for (int attempt = 0; attempt < 10; ++attempt) {
        ++last.attempts;
        const int grow = hint.grow;
        // per-row working rows
        DBuf<int64_t> capb(p), capv(p), boff(p + 1), voff(p + 1);
        const int64_t floor_b = (int64_t)grow * ((A.nb + p - 1) / p), floor_w = (int64_t)grow * ((A.nw + p - 1) / p);
        k_row_caps<<<grid_for(p, 256), 256, 0, s>>>(p, A.rb.p, A.rp.p, A.wp.p, grow, floor_b, floor_w, capb.p, capv.p);
        VB_LAUNCH_CHECK();
        int64_t totb = scan_i64(capb.p, boff.p, p, s);
        int64_t totv = scan_i64(capv.p, voff.p, p, s);
        DBuf<int> wcols(totb), woffs(totb);
        DBuf<unsigned char> west(totb);
        DBuf<T> wvals(totv);
        DBuf<RowState> rs(p);
        DBuf<IlutRowRec> rec(p);
        // the L and U pools are sized from the input matrix; a pool that runs out stops the
        // attempt, which then runs again with larger pools.  A row's L and U output never
        // exceed its working row, so pools as large as all working rows cannot run out:
        // that bounds them.
        const int64_t capb_pool = std::max<int64_t>(
            std::min<int64_t>((int64_t)(hint.pool * (double)A.nb), totb), 64);
        const int64_t capv_pool = std::max<int64_t>(
            std::min<int64_t>((int64_t)(hint.pool * (double)A.nv), totv), (int64_t)64 * A.maxm);
        DBuf<int> lci(capb_pool), lco(capb_pool), uci(capb_pool), uco(capb_pool);
        DBuf<T> lv(capv_pool), uv(capv_pool);
        DBuf<int64_t> cursors(4);
        // LDS of the wave kernel: the largest working-row list this attempt allows
        IlutLds lds;
        lds.maxm = A.maxm;
        // the block list held in LDS: its own capacity, independent of the rows' room in
        // global memory, so that the LDS of a workgroup (and with it the workgroups resident
        // per CU) does not grow with that room
        {
            int cap = std::max(hint.rbcap, 64);
            while (cap < 2 * max_na && cap < kMaxRowBlocks) cap *= 2;
            lds.rbcap = std::min(cap, kMaxRowBlocks);
        }
        // hash load stays below two thirds, and a free slot always ends a probe
        lds.hcap = 64;
        while (2 * lds.hcap < 3 * lds.rbcap) lds.hcap *= 2;
        lds.ustage = kUStage;
        const size_t lds_bytes = ilut_lds_bytes<T>(lds);
        // cnt: three rotating waiting-list counters, two ready counters, finished rows
        DBuf<int> done(p), ready(p), cnt(8);
        DBuf<IlutWait> waits(2 * (size_t)p);
        DBuf<unsigned long long> moved(1);
        fill_val<unsigned long long>(moved.p, 0ull, 1, s);
        VB_HIP(hipMemsetAsync(rs.p, 0, sizeof(RowState) * p, s));
        fill_i64(cursors.p, 0, 4, s);
        fill_i32(done.p, 0, p, s);
        // waiting list of launch 1 (odd launches read the second list)
        k_wait_init<<<grid_for(p, 256), 256, 0, s>>>(p, waits.p + p);
        VB_LAUNCH_CHECK();
        // waiting counts (3), ready counts (2), finished rows, smallest ready row (2)
        const int cnt0[8] = {0, p, 0, 0, 0, 0, INT_MAX, INT_MAX};
        to_device(cnt.p, cnt0, 8, s);
        VB_HIP(hipMemsetAsync(err, 0, 4 * sizeof(int), s));
        int *cw = cnt.p, *cr = cnt.p + 3, *nfin = cnt.p + 5, *mr = cnt.p + 6;
        const unsigned grid = (unsigned)std::min(p, kIlutGrid);
        int finished = 0, launch = 0, code = 0, eblock = 0;
        // Groups of kCheckEvery launches, each followed by a copy of the finished-row count
        // and the error record into pinned memory and an event.  The host queues group g + 1
        // before it waits for the record of group g, so the device never idles on the check;
        // a group queued after the last row finished sees empty lists and does nothing.
        int *hrec = (int *)pinned_staging(2 * 16 * sizeof(int));
        hipEvent_t gev[2] = {nullptr, nullptr};
        VB_HIP(hipEventCreateWithFlags(&gev[0], hipEventDisableTiming));
        VB_HIP(hipEventCreateWithFlags(&gev[1], hipEventDisableTiming));
        struct EvGuard {
            hipEvent_t *e;
            ~EvGuard() {
                (void)hipEventDestroy(e[0]);
                (void)hipEventDestroy(e[1]);
            }
        } evg{gev};
        auto queue_group = [&](int g) {
            for (int q = 0; q < kCheckEvery; ++q) {
                ++launch;
                const IlutWait *w_in = waits.p + (size_t)(launch & 1) * p;
                IlutWait *w_out = waits.p + (size_t)((launch + 1) & 1) * p;
                k_ilut_gather<<<kGatherBlocks, kGatherThreads, 0, s>>>(w_in, cw + launch % 3, done.p, ready.p,
                                                            cr + launch % 2, w_out, cw + (launch + 1) % 3,
                                                            mr + launch % 2);
                VB_LAUNCH_CHECK();
                KScope ks(VBARMS_K_ILUT, 0.0, s);
                k_ilut_wave<T><<<grid, kIlutThreads, lds_bytes, s>>>(
                    launch, p, ready.p, cr + launch % 2, cr + (launch + 1) % 2, mr + launch % 2, mr + (launch + 1) % 2,
                    w_out, cw + (launch + 1) % 3,
                    cw + (launch + 2) % 3, nfin, A.rb.p, A.rp.p, A.ci.p, A.co.p, A.wp.p, A.vp.p, A.v.p,
                    droptol, min_ratio, done.p, rs.p, boff.p, voff.p, wcols.p, woffs.p, west.p, wvals.p, last.dl.p,
                    last.dl_off.p, last.dl_piv.p, rec.p, lci.p, lco.p, lv.p, uci.p, uco.p, uv.p, cursors.p, capb_pool,
                    capv_pool, err, lvl, moved.p, lds);
                VB_LAUNCH_CHECK();
            }
            int *slot = hrec + 16 * (g & 1);
            VB_HIP(hipMemcpyAsync(slot, cnt.p, 6 * sizeof(int), hipMemcpyDeviceToHost, s));
            VB_HIP(hipMemcpyAsync(slot + 8, err, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
            VB_HIP(hipEventRecord(gev[g & 1], s));
        };
        queue_group(0);
        int waves = 0;
        for (int g = 0;; ++g) {
            // every launch finishes at least one row: the smallest unfinished row depends only
            // on rows finished in earlier launches, so the gather always finds it ready, and as
            // the smallest ready row it is exempt from the step cap
            if ((int64_t)g * kCheckEvery > (int64_t)p + kCheckEvery) {
                (void)hipStreamSynchronize(s);
                fail(VBARMS_ERR_HIP, "block ILUT made no progress");
            }
            queue_group(g + 1);
            VB_HIP(hipEventSynchronize(gev[g & 1]));
            const int *slot = hrec + 16 * (g & 1);
            code = slot[8];
            eblock = slot[10];
            waves = (g + 1) * kCheckEvery;
            if (code != 0) break;
            const int now = slot[5];
            if (now < p && now < finished + kCheckEvery) {
                (void)hipStreamSynchronize(s);
                fail(VBARMS_ERR_HIP, "block ILUT made no progress");
            }
            finished = now;
            if (finished >= p) break;
        }
        VB_HIP(hipStreamSynchronize(s));  // the group queued after the last check
        last.waves = waves;
        {
            // the bytes the waves moved, credited to the ILUT timing class
            KTimer *kt = cur_ktimer();
            if (kt && kt->on) kt->tot[VBARMS_K_ILUT].bytes += (double)read_one(moved.p, s);
        }
        if (code == VBARMS_ERR_OOM && attempt < 9) {
            // a working row (eblock >= 0), a pool (eblock == -1) or the LDS block list
            // (eblock <= -2) ran out of room: start again with more, and keep the larger
            // size for the next factorization on this handle
            if (eblock >= 0) hint.grow *= 2;
            else if (eblock == -1) hint.pool *= 2.0;
            else if (lds.rbcap < kMaxRowBlocks) hint.rbcap = 2 * lds.rbcap;
            else fail(VBARMS_ERR_OOM, "a last-level row has more than 1024 blocks");
            continue;
        }
        if (code != 0) return;  // reported by the caller from the error record
        pool_to_panel<T>(p, A.h_rb, A.rb, rec.p, 0, lci.p, lv.p, last.L, s);
        pool_to_panel<T>(p, A.h_rb, A.rb, rec.p, 1, uci.p, uv.p, last.U, s);
        VB_HIP(hipStreamSynchronize(s));
        break;
    }
    // level schedules of the two triangular sweeps
    std::vector<int64_t> rp;
    std::vector<int> ci;
    to_host(rp, last.L.rp.p, p + 1, s);
    to_host(ci, last.L.ci.p, last.L.nb, s);
    level_schedule(p, rp, ci, false, last.lorder, last.lptr);
    to_host(rp, last.U.rp.p, p + 1, s);
    to_host(ci, last.U.ci.p, last.U.nb, s);
    level_schedule(p, rp, ci, true, last.uorder, last.uptr);
    // bytes of the two sweeps: L and U values and column lists, the pivot-block LU
    // factors and pivots, the row offsets, b, t (written and read) and x
    last.sweep_bytes = (double)sizeof(T) * (double)(last.L.nv + last.U.nv + dtot) + 4.0 * (double)(last.L.nw + last.U.nw) +
                       2.0 * 20.0 * (p + 1) + 4.0 * n + 8.0 * 4.0 * n + 8.0 * p;
    // one descriptor per block row, in the order of its sweep
    {
        std::vector<int64_t> hdl, lwp, lvp, uwp, uvp;
        to_host(hdl, last.dl_off.p, p + 1, s);
        to_host(lwp, last.L.wp.p, p + 1, s);
        to_host(lvp, last.L.vp.p, p + 1, s);
        to_host(uwp, last.U.wp.p, p + 1, s);
        to_host(uvp, last.U.vp.p, p + 1, s);
        const std::vector<int> &rbh = A.h_rb;
        std::vector<SweepRow> lr(p), ur(p);
        for (int q = 0; q < p; ++q) {
            const int i = last.lorder[q];
            lr[q] = SweepRow{i, rbh[i], rbh[i + 1] - rbh[i], 0, lwp[i], lwp[i + 1] - lwp[i], lvp[i], hdl[i]};
            const int j = last.uorder[q];
            ur[q] = SweepRow{j, rbh[j], rbh[j + 1] - rbh[j], 0, uwp[j], uwp[j + 1] - uwp[j], uvp[j], hdl[j]};
        }
        const size_t words = sizeof(SweepRow) / sizeof(int64_t);
        last.d_lrows.alloc((size_t)p * words);
        last.d_urows.alloc((size_t)p * words);
        to_device((SweepRow *)last.d_lrows.p, lr.data(), p, s);
        to_device((SweepRow *)last.d_urows.p, ur.data(), p, s);
        VB_HIP(hipStreamSynchronize(s));  // the host vectors are the copy sources
    }
    VB_HIP(hipStreamSynchronize(s));
}

// the level launches of both sweeps for nv vectors (n apart): t = L^{-1} b, then
// x = U^{-1} t (pivot blocks included); t holds nv vectors
template <class T>
static void sweep_launches(LastLevel<T> &last, const double *b, double *x, double *t, int nv, hipStream_t s) {
    const Panel<T> &L = last.L, &U = last.U;
    const SweepRow *lrows = (const SweepRow *)last.d_lrows.p, *urows = (const SweepRow *)last.d_urows.p;
    const int64_t n = last.A.h_rb.back();
    for (size_t l = 0; l + 1 < last.lptr.size(); ++l) {
        int cnt = last.lptr[l + 1] - last.lptr[l];
        k_trsv_level<T><<<dim3(cnt, nv), kSweepThreads, 0, s>>>(lrows + last.lptr[l], 0, L.sc.p, L.v.p, last.dl.p,
                                                                last.dl_piv.p, b, t, n);
        VB_LAUNCH_CHECK();
    }
    for (size_t l = 0; l + 1 < last.uptr.size(); ++l) {
        int cnt = last.uptr[l + 1] - last.uptr[l];
        k_trsv_level<T><<<dim3(cnt, nv), kSweepThreads, 0, s>>>(urows + last.uptr[l], 1, U.sc.p, U.v.p, last.dl.p,
                                                                last.dl_piv.p, t, x, n);
        VB_LAUNCH_CHECK();
    }
}

// Records the sweeps for nv vectors once on a private stream into g; the graph reads gb
// and writes gx (nv vectors each), with t as its workspace.
template <class T>
static void capture_sweeps(LastLevel<T> &last, int nv, LaunchGraph &g, DBuf<double> &gb, DBuf<double> &gx,
                           DBuf<double> &t) {
    const int64_t n = last.A.h_rb.back();
    g.reset();
    gb.alloc((size_t)std::max<int64_t>(n, 1) * nv);
    gx.alloc((size_t)std::max<int64_t>(n, 1) * nv);
    if (nv > 1) t.alloc((size_t)std::max<int64_t>(n, 1) * nv);
    hipStream_t cs = nullptr;
    VB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
        try {
            sweep_launches<T>(last, gb.p, gx.p, t.p, nv, cs);
        } catch (...) {
            hipGraph_t gr = nullptr;
            (void)hipStreamEndCapture(cs, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            (void)hipStreamDestroy(cs);
            throw;
        }
        e = hipStreamEndCapture(cs, &g.graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        g.reset();
        fail(VBARMS_ERR_HIP, std::string("capturing the last-level sweeps: ") + hipGetErrorString(e));
    }
}

template <class T>
void solve_last(LastLevel<T> &last, const double *b, double *x, int *err, hipStream_t s, int nv) {
    (void)err;
    const int p = last.A.p;
    if (p == 0 || nv < 1) return;
    const int64_t n = last.A.h_rb.back();
    if (!last.use_graph) {
        KScope ks(VBARMS_K_TRSV, last.sweep_bytes * nv, s);
        if (nv > 1 && last.t_mv.n < (size_t)n * nv) last.t_mv.alloc((size_t)n * nv);
        sweep_launches<T>(last, b, x, nv == 1 ? last.t.p : last.t_mv.p, nv, s);
        return;
    }
    LaunchGraph &g = nv == 1 ? last.sweeps : last.sweeps_mv;
    DBuf<double> &gb = nv == 1 ? last.gb : last.gb_mv, &gx = nv == 1 ? last.gx : last.gx_mv;
    if (nv == 1 && !g.exec) capture_sweeps<T>(last, 1, g, gb, gx, last.t);
    if (nv > 1 && (!g.exec || last.mv_nv != nv)) {
        capture_sweeps<T>(last, nv, g, gb, gx, last.t_mv);
        last.mv_nv = nv;
    }
    KScope ks(VBARMS_K_TRSV, last.sweep_bytes * nv, s);
    const size_t bytes = sizeof(double) * (size_t)n * nv;
    if (b != gb.p) VB_HIP(hipMemcpyAsync(gb.p, b, bytes, hipMemcpyDeviceToDevice, s));
    VB_HIP(hipGraphLaunch(g.exec, s));
    if (x != gx.p) VB_HIP(hipMemcpyAsync(x, gx.p, bytes, hipMemcpyDeviceToDevice, s));
}

template void factor_last<double>(LastLevel<double> &, double, double, int, IlutHint &, int *, hipStream_t);
template void factor_last<float>(LastLevel<float> &, double, double, int, IlutHint &, int *, hipStream_t);
template void solve_last<double>(LastLevel<double> &, const double *, double *, int *, hipStream_t, int);
template void solve_last<float>(LastLevel<float> &, const double *, double *, int *, hipStream_t, int);

}  // namespace vb
