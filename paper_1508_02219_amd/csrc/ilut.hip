// Last-level block ILUT (Sec. 3, Alg. 3, IKJ order) and its triangular solves.
//
// Factorization: a persistent kernel whose workgroups take block rows in ascending order
// from a ticket counter.  Row i is eliminated against the finished rows k < i present in
// its working row, smallest k first (fill included), exactly like the sequential IKJ
// loop; before using row k it waits for row k's completion flag.  Because rows are
// ticketed in ascending order, every row waited on is already owned by a running
// workgroup, so the waits always end.  The working row lives in an LDS hash map
// (block column -> list slot) with its dense blocks in a per-workgroup global scratch.
// Finished rows are appended to L/U pools and compacted into panels afterwards.
//
// Solves: sync-free block substitution, one wavefront per block row taken in dependency
// order from a ticket counter (ascending for L, descending for U), each waiting on the
// completion flags of the rows it reads.
//
// Every wait has an abort flag and a wall-clock limit, so a fault in the dependency data
// ends the kernel with an error instead of a hang.
#include <algorithm>
#include <climits>

#include "factor.h"

namespace vb {

namespace {

constexpr int kIlutThreads = 256;
constexpr int kCapB = 1024;       // blocks in one working row
constexpr int kHashCap = 2048;    // LDS hash slots (power of two, > 2 kCapB / 2)

struct IlutRowRec {
    int64_t lb, lv, ub, uv;  // block / value offsets in the pools
    int lc, lw, uc, uw;      // block counts and panel widths
};

__device__ inline int h_find(const int *keys, const int *vals, int key) {
    unsigned h = ((unsigned)key * 2654435761u) & (kHashCap - 1);
    for (;;) {
        int k = keys[h];
        if (k == key) return vals[h];
        if (k == -1) return -1;
        h = (h + 1) & (kHashCap - 1);
    }
}
__device__ inline void h_insert(int *keys, int *vals, int key, int val) {
    unsigned h = ((unsigned)key * 2654435761u) & (kHashCap - 1);
    for (;;) {
        int old = atomicCAS(&keys[h], -1, key);
        if (old == -1 || old == key) { vals[h] = val; return; }
        h = (h + 1) & (kHashCap - 1);
    }
}

__device__ inline bool wait_flag(const int *flag, int epoch, int *abort, int *err, unsigned long long limit, int row) {
    unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() - t0 > limit) {
            dev_set_error(err, VBARMS_ERR_HIP, 1000, row);
            __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

template <class T>
__global__ void __launch_bounds__(kIlutThreads) k_ilut(
    int p, const int *rb, const int64_t *rp, const int *ci, const int *co, const int64_t *wp, const int64_t *vp,
    const T *av, double droptol, int *ticket, int *done, int epoch, int *abort, int *err, unsigned long long limit,
    T *scratch, int64_t capv, T *dl, const int64_t *dl_off, int *dl_piv, IlutRowRec *rec, int *lci, int *lco, T *lv,
    int *uci, int *uco, T *uv, int64_t *cursors, int64_t capb_pool, int64_t capv_pool, int lvl) {
    __shared__ int hkeys[kHashCap], hvals[kHashCap];
    __shared__ int wcol[kCapB];
    __shared__ int woff[kCapB];
    __shared__ unsigned char wst[kCapB];  // 0 pending, 1 eliminated, 2 dropped
    __shared__ int s_row, s_n, s_used, s_min, s_flag, s_abort;
    __shared__ int s_lc, s_lw, s_uc, s_uw;
    __shared__ int64_t s_lb, s_lv, s_ub, s_uv;
    const int t = threadIdx.x;
    T *w = scratch + (int64_t)blockIdx.x * capv;

    for (;;) {
        if (t == 0) s_row = atomicAdd(ticket, 1);
        __syncthreads();
        const int i = s_row;
        if (i >= p) break;
        const int m = rb[i + 1] - rb[i];
        for (int h = t; h < kHashCap; h += kIlutThreads) hkeys[h] = -1;
        if (t == 0) {
            int nA = (int)(rp[i + 1] - rp[i]);
            s_abort = __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (nA > kCapB || (int64_t)m * (wp[i + 1] - wp[i]) > capv) {
                dev_set_error(err, VBARMS_ERR_OOM, lvl, i);
                __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_abort = 1;
            }
            s_n = nA;
            s_used = (int)(m * (wp[i + 1] - wp[i]));
        }
        __syncthreads();
        if (!s_abort) {
            // load row i: list slot e = block e of the row, blocks stored contiguously
            const int64_t b0 = rp[i];
            for (int e = t; e < s_n; e += kIlutThreads) {
                wcol[e] = ci[b0 + e];
                woff[e] = m * co[b0 + e];
                wst[e] = 0;
                h_insert(hkeys, hvals, ci[b0 + e], e);
            }
            const int64_t W = wp[i + 1] - wp[i];
            const T *A = av + vp[i];
            for (int64_t c = t; c < W; c += kIlutThreads) {
                int64_t b = dev_floor32(co, b0, rp[i + 1], (int)c);
                int nJ = (b + 1 < rp[i + 1] ? co[b + 1] : (int)W) - co[b];
                int local = (int)(c - co[b]);
                int off = m * co[b];
                for (int r = 0; r < m; ++r) w[off + r * nJ + local] = A[r * W + c];
            }
        }
        __syncthreads();
        int last_k = -1;
        while (!s_abort) {
            if (t == 0) s_min = INT_MAX;
            __syncthreads();
            for (int e = t; e < s_n; e += kIlutThreads) {
                int K = wcol[e];
                if (K < i && K > last_k && wst[e] == 0) atomicMin(&s_min, K);
            }
            __syncthreads();
            const int k = s_min;
            if (k == INT_MAX) break;
            last_k = k;
            const int ek = h_find(hkeys, hvals, k);
            if (t == 0) {
                if (!wait_flag(&done[k], epoch, abort, err, limit, i)) s_abort = 1;
            }
            __syncthreads();
            if (s_abort) break;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int mk = rb[k + 1] - rb[k];
            const IlutRowRec rk = rec[k];
            // row k's record must describe pool ranges; anything else is reported, not used
            if (t == 0) {
                bool ok = ek >= 0 && ek < s_n && rk.uc >= 0 && rk.ub >= 0 && rk.ub + rk.uc <= capb_pool &&
                          rk.uw >= 0 && rk.uv >= 0 && rk.uv + (int64_t)mk * rk.uw <= capv_pool &&
                          (rk.uc == 0) == (rk.uw == 0);
                for (int q = 0; q < mk; ++q) {
                    int pq = dl_piv[rb[k] + q];
                    ok = ok && pq >= q && pq < mk;
                }
                if (!ok) {
                    dev_set_error(err, VBARMS_ERR_HIP, 3001, i);
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_abort = 1;
                }
            }
            __syncthreads();
            if (s_abort) break;
            T *M = w + woff[ek];
            const T *dk = dl + dl_off[k];
            if (t < m) {
                dev_row_solve_u<T>(mk, dk, M + t * mk, 1);
                dev_row_solve_lp<T>(mk, dk, dl_piv + rb[k], M + t * mk, 1);
            }
            __syncthreads();
            if (t == 0) s_flag = dev_drop<T>(m, mk, M, mk, droptol);
            __syncthreads();
            if (s_flag) {
                if (t == 0) wst[ek] = 2;
                __syncthreads();
                continue;
            }
            if (t == 0) wst[ek] = 1;
            // fill: blocks of U row k not yet in the working row
            for (int b = t; b < rk.uc; b += kIlutThreads) {
                int J = uci[rk.ub + b];
                if (J <= k || J >= p) {
                    dev_set_error(err, VBARMS_ERR_HIP, 3002, i);
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_abort = 1;
                    continue;
                }
                if (h_find(hkeys, hvals, J) >= 0) continue;
                int nJ = rb[J + 1] - rb[J];
                int e = atomicAdd(&s_n, 1);
                int off = atomicAdd(&s_used, m * nJ);
                if (e >= kCapB || (int64_t)off + m * nJ > capv) {
                    dev_set_error(err, VBARMS_ERR_OOM, lvl, i);
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_abort = 1;
                    continue;
                }
                wcol[e] = J;
                woff[e] = off;
                wst[e] = 0;
                for (int q = 0; q < m * nJ; ++q) w[off + q] = T(0);
                h_insert(hkeys, hvals, J, e);
            }
            __syncthreads();
            if (s_abort) break;
            // w_J -= M U_kJ for every block J of U row k
            const T *U = uv + rk.uv;
            const int UW = rk.uw;
            for (int c = t; c < UW; c += kIlutThreads) {
                int64_t b = dev_floor32(uco, rk.ub, rk.ub + rk.uc, c);
                int J = uci[b];
                int nJ = rb[J + 1] - rb[J];
                int local = c - uco[b];
                int e = h_find(hkeys, hvals, J);
                if (e < 0 || local < 0 || local >= nJ) {
                    dev_set_error(err, VBARMS_ERR_HIP, 3003, i);
                    continue;
                }
                T *wj = w + woff[e] + local;
                for (int r = 0; r < m; ++r) {
                    T acc = wj[r * nJ];
                    for (int q = 0; q < mk; ++q) acc = acc - M[r * mk + q] * U[q * UW + c];
                    wj[r * nJ] = acc;
                }
            }
            __syncthreads();
        }
        __syncthreads();
        // finalize row i
        if (!s_abort) {
            if (t == 0) {
                s_lc = s_lw = s_uc = s_uw = 0;
                int ei = h_find(hkeys, hvals, i);
                T *d = dl + dl_off[i];
                if (ei < 0) {
                    dev_set_error(err, VBARMS_ERR_SINGULAR, lvl, i);
                    for (int q = 0; q < m * m; ++q) d[q] = T(0);
                } else {
                    for (int q = 0; q < m * m; ++q) d[q] = w[woff[ei] + q];
                    if (!dev_gepp<T>(m, d, dl_piv + rb[i])) dev_set_error(err, VBARMS_ERR_SINGULAR, lvl, i);
                }
            }
            // classify entries: keep flag in wst (3 = kept L, 4 = kept U, else discarded)
            for (int e = t; e < s_n; e += kIlutThreads) {
                int K = wcol[e];
                int nK = rb[K + 1] - rb[K];
                if (K < i) {
                    wst[e] = wst[e] == 1 ? 3 : 0;
                } else if (K > i) {
                    wst[e] = dev_drop<T>(m, nK, w + woff[e], nK, droptol) ? 0 : 4;
                } else {
                    wst[e] = 0;
                }
            }
            __syncthreads();
            for (int e = t; e < s_n; e += kIlutThreads) {
                int K = wcol[e];
                int nK = rb[K + 1] - rb[K];
                if (wst[e] == 3) { atomicAdd(&s_lc, 1); atomicAdd(&s_lw, nK); }
                if (wst[e] == 4) { atomicAdd(&s_uc, 1); atomicAdd(&s_uw, nK); }
            }
            __syncthreads();
            if (t == 0) {
                s_lb = atomicAdd((unsigned long long *)&cursors[0], (unsigned long long)s_lc);
                s_lv = atomicAdd((unsigned long long *)&cursors[1], (unsigned long long)m * s_lw);
                s_ub = atomicAdd((unsigned long long *)&cursors[2], (unsigned long long)s_uc);
                s_uv = atomicAdd((unsigned long long *)&cursors[3], (unsigned long long)m * s_uw);
                if (s_lb + s_lc > capb_pool || s_lv + (int64_t)m * s_lw > capv_pool || s_ub + s_uc > capb_pool ||
                    s_uv + (int64_t)m * s_uw > capv_pool) {
                    dev_set_error(err, VBARMS_ERR_OOM, lvl, -1);
                    __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_abort = 1;
                }
            }
            __syncthreads();
            if (!s_abort) {
                // output position = rank by block column; panel offset = widths of smaller columns
                for (int e = t; e < s_n; e += kIlutThreads) {
                    int st = wst[e];
                    if (st != 3 && st != 4) continue;
                    int K = wcol[e];
                    int rank = 0, off = 0;
                    for (int f = 0; f < s_n; ++f) {
                        if (wst[f] == st && wcol[f] < K) {
                            ++rank;
                            off += rb[wcol[f] + 1] - rb[wcol[f]];
                        }
                    }
                    int nK = rb[K + 1] - rb[K];
                    const T *src = w + woff[e];
                    if (st == 3) {
                        lci[s_lb + rank] = K;
                        lco[s_lb + rank] = off;
                        for (int r = 0; r < m; ++r)
                            for (int c = 0; c < nK; ++c) lv[s_lv + (int64_t)r * s_lw + off + c] = src[r * nK + c];
                    } else {
                        uci[s_ub + rank] = K;
                        uco[s_ub + rank] = off;
                        for (int r = 0; r < m; ++r)
                            for (int c = 0; c < nK; ++c) uv[s_uv + (int64_t)r * s_uw + off + c] = src[r * nK + c];
                    }
                }
                if (t == 0) rec[i] = IlutRowRec{s_lb, s_lv, s_ub, s_uv, s_lc, s_lw, s_uc, s_uw};
            }
        }
        if (s_abort && t == 0) rec[i] = IlutRowRec{0, 0, 0, 0, 0, 0, 0, 0};
        __threadfence();
        __syncthreads();
        if (t == 0) __hip_atomic_store(&done[i], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void k_rec_counts(int p, const IlutRowRec *rec, int which, int64_t *cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    cnt[i] = which == 0 ? rec[i].lc : rec[i].uc;
}
// copy pool rows into ordered block-column lists
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

unsigned long long wall_ticks_per_second() {
    static unsigned long long hz = 0;
    if (!hz) {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            hz = (unsigned long long)khz * 1000ull;
        else
            hz = 100000000ull;
    }
    return hz;
}

// ---- sync-free block substitution ------------------------------------------------------
constexpr int kSolveTG = 8;  // lanes per scalar row

// mode 0: t_i = b_i - sum_k L_ik t_k (ascending); mode 1: x_i = D_i^{-1}(t_i - sum_j U_ij x_j)
template <class T>
__global__ void __launch_bounds__(256) k_block_trsv(int p, int mode, const int *rb, const int64_t *rp, const int *ci,
                                                    const int64_t *wp, const int64_t *vp, const int *sc, const T *v,
                                                    const T *dl, const int64_t *dl_off, const int *dl_piv,
                                                    const double *b, double *x, int *ticket, int *done, int epoch,
                                                    int *abort, int *err, unsigned long long limit) {
    __shared__ double sv[4][VBARMS_MAX_BLOCK];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int grp = lane / kSolveTG, gl = lane % kSolveTG;
    for (;;) {
        int tk = 0;
        if (lane == 0) tk = atomicAdd(ticket, 1);
        tk = __shfl(tk, 0);
        if (tk >= p) return;
        const int i = mode == 0 ? tk : p - 1 - tk;
        const int m = rb[i + 1] - rb[i];
        // wait for every row this one reads
        for (int64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) {
            int K = ci[k];
            if (K < 0 || K >= p || (mode == 0 ? K >= i : K <= i)) {
                dev_set_error(err, VBARMS_ERR_HIP, 3004, i);
                __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                continue;
            }
            wait_flag(&done[K], epoch, abort, err, limit, i);
        }
        __builtin_amdgcn_wave_barrier();  // every lane has seen all its flags
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int64_t W = wp[i + 1] - wp[i];
        for (int r0 = 0; r0 < m; r0 += 64 / kSolveTG) {
            const int r = r0 + grp;
            double acc = 0.0;
            if (r < m) {
                const T *a = v + vp[i] + (int64_t)r * W;
                const int *c = sc + wp[i];
                for (int64_t j = gl; j < W; j += kSolveTG) acc += (double)a[j] * x[c[j]];
            }
#pragma unroll
            for (int off = kSolveTG / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kSolveTG);
            if (r < m && gl == 0) sv[wv][r] = b[rb[i] + r] - acc;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (lane == 0) {
            double *y = sv[wv];
            if (mode == 1) {
                const T *d = dl + dl_off[i];
                dev_lu_fwd<T, double>(m, d, dl_piv + rb[i], y);
                dev_lu_bwd<T, double>(m, d, y);
            }
            for (int r = 0; r < m; ++r) x[rb[i] + r] = y[r];
            __threadfence();
            __hip_atomic_store(&done[i], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __builtin_amdgcn_wave_barrier();  // sv[wv] is reused by the next row
    }
}

// number of persistent workgroups / wavefronts (tuning knobs; 1 serializes the sweep)
int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    int x = atoi(v);
    return x > 0 ? x : dflt;
}

}  // namespace

template <class T>
void factor_last(LastLevel<T> &last, double droptol, int lvl, int *err, hipStream_t s) {
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
    last.done_f.alloc(std::max(p, 1));
    last.done_b.alloc(std::max(p, 1));
    fill_i32(last.done_f.p, 0, p, s);
    fill_i32(last.done_b.p, 0, p, s);
    last.tickets.alloc(4);
    last.t.alloc(std::max(n, 1));
    last.epoch = 0;
    if (p == 0) {
        panel_set_blocks(last.L, A.h_rb, A.h_rb, s);
        panel_set_blocks(last.U, A.h_rb, A.h_rb, s);
        last.L.rp.alloc(1); fill_i64(last.L.rp.p, 0, 1, s); panel_finish_layout(last.L, s);
        last.U.rp.alloc(1); fill_i64(last.U.rp.p, 0, 1, s); panel_finish_layout(last.U, s);
        return;
    }
    // pools sized generously from the input (fill grows rows); overflow is reported as OOM
    const int maxm = A.maxm;
    int64_t capb_pool = std::max<int64_t>(4 * A.nb + 1024, 4096);
    int64_t capv_pool = std::max<int64_t>(4 * A.nv + 1024, 65536);
    int nslot = std::min(p, env_int("VBARMS_ILUT_WORKGROUPS", 1024));
    // working-row capacity: generous multiple of the largest input row, bounded by the
    // largest row the LDS list can describe
    std::vector<int64_t> hvp;
    to_host(hvp, A.vp.p, p + 1, s);
    int64_t maxrow = 0;
    for (int i = 0; i < p; ++i) maxrow = std::max(maxrow, hvp[i + 1] - hvp[i]);
    int64_t capv = std::min<int64_t>((int64_t)kCapB * maxm * maxm, std::max<int64_t>(65536, 16 * maxrow));
    for (int attempt = 0; attempt < 3; ++attempt) {
        DBuf<T> scratch((size_t)nslot * capv);
        DBuf<IlutRowRec> rec(p);
        DBuf<int> lci(capb_pool), lco(capb_pool), uci(capb_pool), uco(capb_pool);
        DBuf<T> lv(capv_pool), uv(capv_pool);
        DBuf<int64_t> cursors(4);
        DBuf<int> abort(1), done(p);
        fill_i64(cursors.p, 0, 4, s);
        fill_i32(abort.p, 0, 1, s);
        fill_i32(done.p, 0, p, s);
        fill_i32(last.tickets.p, 0, 4, s);
        VB_HIP(hipMemsetAsync(err, 0, 4 * sizeof(int), s));
        unsigned long long limit = 20ull * wall_ticks_per_second();
        k_ilut<T><<<nslot, kIlutThreads, 0, s>>>(p, A.rb.p, A.rp.p, A.ci.p, A.co.p, A.wp.p, A.vp.p, A.v.p, droptol,
                                                   last.tickets.p, done.p, 1, abort.p, err, limit, scratch.p, capv,
                                                   last.dl.p, last.dl_off.p, last.dl_piv.p, rec.p, lci.p, lco.p, lv.p,
                                                   uci.p, uco.p, uv.p, cursors.p, capb_pool, capv_pool, lvl);
        VB_LAUNCH_CHECK();
        std::vector<int> herr;
        to_host(herr, err, 4, s);
        if (herr[0] == VBARMS_ERR_OOM && herr[2] == -1 && attempt < 2) {
            capb_pool *= 3;
            capv_pool *= 3;
            continue;  // pools too small: retry with larger pools
        }
        if (herr[0] != 0) return;
        pool_to_panel<T>(p, A.h_rb, A.rb, rec.p, 0, lci.p, lv.p, last.L, s);
        pool_to_panel<T>(p, A.h_rb, A.rb, rec.p, 1, uci.p, uv.p, last.U, s);
        return;
    }
}

template <class T>
void solve_last(LastLevel<T> &last, const double *b, double *x, int *err, hipStream_t s) {
    const int p = last.A.p;
    if (p == 0) return;
    ++last.epoch;
    if (last.epoch == INT_MAX) {
        fill_i32(last.done_f.p, 0, p, s);
        fill_i32(last.done_b.p, 0, p, s);
        last.epoch = 1;
    }
    fill_i32(last.tickets.p, 0, 4, s);  // two tickets, tickets[2] = abort flag
    unsigned long long limit = 10ull * wall_ticks_per_second();
    // persistent wavefronts, four per workgroup; a wave waits only on rows ticketed before it
    const int waves = std::min(p, env_int("VBARMS_TRSV_WAVES", 4096));
    const int threads = waves >= 4 ? 256 : 64 * waves;
    const unsigned blocks = grid_for((int64_t)waves * 64, threads);
    const Panel<T> &L = last.L, &U = last.U;
    k_block_trsv<T><<<blocks, threads, 0, s>>>(p, 0, L.rb.p, L.rp.p, L.ci.p, L.wp.p, L.vp.p, L.sc.p, L.v.p,
                                               last.dl.p, last.dl_off.p, last.dl_piv.p, b, last.t.p, last.tickets.p,
                                               last.done_f.p, last.epoch, last.tickets.p + 2, err, limit);
    VB_LAUNCH_CHECK();
    k_block_trsv<T><<<blocks, threads, 0, s>>>(p, 1, U.rb.p, U.rp.p, U.ci.p, U.wp.p, U.vp.p, U.sc.p, U.v.p,
                                               last.dl.p, last.dl_off.p, last.dl_piv.p, last.t.p, x,
                                               last.tickets.p + 1, last.done_b.p, last.epoch, last.tickets.p + 2, err,
                                               limit);
    VB_LAUNCH_CHECK();
}

template void factor_last<double>(LastLevel<double> &, double, int, int *, hipStream_t);
template void factor_last<float>(LastLevel<float> &, double, int, int *, hipStream_t);
template void solve_last<double>(LastLevel<double> &, const double *, double *, int *, hipStream_t);
template void solve_last<float>(LastLevel<float> &, const double *, double *, int *, hipStream_t);

}  // namespace vb
