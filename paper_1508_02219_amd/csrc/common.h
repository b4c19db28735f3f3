// Internal declarations shared by the VBARMS HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <memory>
#include <string>
#include <vector>

#include "../../include/vbarms.h"

namespace vb {

// ---------------------------------------------------------------------------------
// Errors: internal code throws VbError; the C ABI converts it to a return code.
// ---------------------------------------------------------------------------------
struct VbError {
    int code;
    std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw VbError{code, msg}; }

#define VB_HIP(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            ::vb::fail(e_ == hipErrorOutOfMemory ? VBARMS_ERR_OOM : VBARMS_ERR_HIP,          \
                       std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    } while (0)

#define VB_LAUNCH_CHECK() VB_HIP(hipGetLastError())

// ---------------------------------------------------------------------------------
// Device buffers
//
// Every buffer is allocated and freed in stream order on the stream of the API call in
// progress (cur_stream()), so a buffer that goes out of scope is released only after
// every kernel enqueued before the release has finished with it.
// ---------------------------------------------------------------------------------
inline hipStream_t &cur_stream() {
    static thread_local hipStream_t s = nullptr;
    return s;
}
struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t s) : prev(cur_stream()) { cur_stream() = s; }
    ~StreamScope() { cur_stream() = prev; }
};

// ---------------------------------------------------------------------------------
// Optional timing of kernel classes: a pair of events recorded on the launch stream
// around each timed launch; the pairs are read after the stream has synchronized.
// ---------------------------------------------------------------------------------
struct KTimer {
    struct Pair {
        hipEvent_t a, b;
        int cls;
        double bytes;
    };
    bool on = false;
    std::vector<Pair> pend;
    std::vector<hipEvent_t> spare;
    vbarms_kstat tot[VBARMS_K_COUNT] = {};
    hipEvent_t take() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // call only after the stream of every pending pair has synchronized
    void resolve() {
        for (const Pair &q : pend) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
                tot[q.cls].calls += 1;
                tot[q.cls].ms += ms;
                tot[q.cls].bytes += q.bytes;
            }
            spare.push_back(q.a);
            spare.push_back(q.b);
        }
        pend.clear();
    }
    void reset() {
        resolve();
        for (auto &t : tot) t = vbarms_kstat{};
    }
    ~KTimer() {
        for (const Pair &q : pend) {
            (void)hipEventDestroy(q.a);
            (void)hipEventDestroy(q.b);
        }
        for (hipEvent_t e : spare) (void)hipEventDestroy(e);
    }
};
inline KTimer *&cur_ktimer() {
    static thread_local KTimer *t = nullptr;
    return t;
}
// Times the launches enqueued during its lifetime as one call of class `cls`.
struct KScope {
    KTimer *t = nullptr;
    hipEvent_t a = nullptr;
    hipStream_t s;
    int cls;
    double bytes;
    KScope(int cls_, double bytes_, hipStream_t s_) : s(s_), cls(cls_), bytes(bytes_) {
        KTimer *k = cur_ktimer();
        if (k && k->on) {
            a = k->take();
            if (a && hipEventRecord(a, s) == hipSuccess) t = k;
        }
    }
    ~KScope() {
        if (!t) return;
        hipEvent_t b = t->take();
        if (b && hipEventRecord(b, s) == hipSuccess) t->pend.push_back(KTimer::Pair{a, b, cls, bytes});
        else t->spare.push_back(a);
    }
    KScope(const KScope &) = delete;
    KScope &operator=(const KScope &) = delete;
};

// Device memory comes from a caching allocator kept per stream (util.hip).  A block
// released on stream s goes back to that stream's free list and is handed out again only
// to work enqueued later on s, so stream order alone makes the reuse safe; no block is
// returned to the runtime while the process runs (except to retry a failed allocation),
// so a steady stream of factorizations of one matrix allocates nothing after the first.
void *dev_alloc(size_t bytes, hipStream_t s);  // throws VbError(OOM)
void dev_free(void *p, hipStream_t s);
struct DevCacheStats {
    size_t live_bytes, cached_bytes, peak_bytes;
    int64_t runtime_allocs;  // calls that reached hipMalloc
};
DevCacheStats dev_cache_stats();
// Pinned host staging memory of at least `bytes`, owned by the calling host thread and kept
// (grown, never shrunk) until the process ends; valid until the thread's next call.
void *pinned_staging(size_t bytes);

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        n = count;
        if (count) {
            try {
                p = (T *)dev_alloc(count * sizeof(T), cur_stream());
            } catch (...) {
                p = nullptr;
                n = 0;
                throw;
            }
        }
    }
    // grow-only reallocation (contents are not preserved)
    void reserve(size_t count) {
        if (count > n) alloc(count);
    }
    void release() {
        if (p) dev_free(p, cur_stream());
        p = nullptr;
        n = 0;
    }
    T *get() const { return p; }
};

template <class T>
inline void to_host(std::vector<T> &dst, const T *src, size_t count, hipStream_t s) {
    dst.resize(count);
    if (count) VB_HIP(hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s));
    VB_HIP(hipStreamSynchronize(s));
}
template <class T>
inline T read_one(const T *src, hipStream_t s) {
    T v{};
    VB_HIP(hipMemcpyAsync(&v, src, sizeof(T), hipMemcpyDeviceToHost, s));
    VB_HIP(hipStreamSynchronize(s));
    return v;
}
template <class T>
inline void to_device(T *dst, const T *src, size_t count, hipStream_t s) {
    if (count) VB_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
}

inline unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > 0x7fffffff) g = 0x7fffffff;
    return (unsigned)g;
}

// ---------------------------------------------------------------------------------
// Block-row panel storage of a variable-block sparse matrix.
//
// Block row I (height m_I = rb[I+1] - rb[I]) owns the blocks k in [rp[I], rp[I+1]) with
// ascending block columns ci[k].  Its values form one dense row-major panel of m_I rows
// and W_I = wp[I+1] - wp[I] columns at v + vp[I]; block k occupies panel columns
// [co[k], co[k] + n_ci[k]).  sc[wp[I] + c] is the scalar column of panel column c, so a
// scalar row of the panel is a CSR row whose column list is shared by the m_I rows of
// its block row.
// ---------------------------------------------------------------------------------
template <class T>
struct Panel {
    int p = 0, q = 0;          // block rows, block columns
    int64_t nb = 0, nw = 0, nv = 0;
    int maxm = 0;              // largest row block
    std::vector<int> h_rb, h_cb;
    DBuf<int> rb, cb;          // [p+1], [q+1]
    DBuf<int64_t> rp, wp, vp;  // [p+1]
    DBuf<int> ci, co;          // [nb]
    DBuf<int> sc;              // [nw]
    DBuf<int> rowblk;          // [n] block row of every scalar row
    DBuf<T> v;                 // [nv]
    int tg = 8;                // lanes per scalar row of the product kernel (autotuned)
};

// Raw view passed to kernels
template <class T>
struct PanelView {
    int p;
    const int *rb, *cb;
    const int64_t *rp, *wp, *vp;
    const int *ci, *co, *sc, *rowblk;
    T *v;
};
template <class T>
inline PanelView<T> view(const Panel<T> &a) {
    return PanelView<T>{a.p, a.rb.p, a.cb.p, a.rp.p, a.wp.p, a.vp.p, a.ci.p, a.co.p, a.sc.p, a.rowblk.p, a.v.p};
}

// ---------------------------------------------------------------------------------
// Device-side helpers
// ---------------------------------------------------------------------------------
// Binary search for `key` in sorted a[lo, hi); returns index or -1.
__device__ inline int64_t dev_find(const int *a, int64_t lo, int64_t hi, int key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        int v = a[mid];
        if (v < key) lo = mid + 1;
        else if (v > key) hi = mid;
        else return mid;
    }
    return -1;
}
// Largest index k in [lo, hi) with a[k] <= key (a sorted ascending, a[lo] <= key).
__device__ inline int64_t dev_floor(const int64_t *a, int64_t lo, int64_t hi, int64_t key) {
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid;
        else hi = mid;
    }
    return lo;
}
__device__ inline int64_t dev_floor32(const int *a, int64_t lo, int64_t hi, int key) {
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Records the first error (code, a, b) in the 4-int device error record.
__device__ inline void dev_set_error(int *err, int code, int a, int b) {
    if (atomicCAS(err, 0, code) == 0) {
        err[1] = a;
        err[2] = b;
    }
}

// The dense per-block kernels below restate the oracle's operation order exactly so that
// FP64 results agree to the last bit when the library is compiled without contraction.

// GEPP in place on an m x m row-major block (first row of maximal magnitude is the pivot).
template <class T>
__device__ inline bool dev_gepp(int m, T *a, int *piv) {
    for (int k = 0; k < m; ++k) {
        int pr = k;
        T amax = fabs(a[k * m + k]);
        for (int r = k + 1; r < m; ++r) {
            T v = fabs(a[r * m + k]);
            if (v > amax) { amax = v; pr = r; }
        }
        piv[k] = pr;
        if (amax == T(0)) return false;
        if (pr != k)
            for (int c = 0; c < m; ++c) { T t = a[k * m + c]; a[k * m + c] = a[pr * m + c]; a[pr * m + c] = t; }
        for (int r = k + 1; r < m; ++r) {
            a[r * m + k] = a[r * m + k] / a[k * m + k];
            T l = a[r * m + k];
            for (int c = k + 1; c < m; ++c) a[r * m + c] = a[r * m + c] - l * a[k * m + c];
        }
    }
    return true;
}
// Barrier of one wavefront: its LDS and memory operations issued so far are visible to
// its other lanes.
__device__ inline void wave_sync() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
// dev_gepp by one wavefront (all 64 lanes call it; m <= 64) on the row-major block a in
// LDS, pivots in pv (LDS).  The pivot search is a wavefront reduction that picks the row
// the sequential scan picks (the first row of largest modulus, the diagonal kept on ties;
// a NaN never wins and a NaN diagonal keeps its row), and every element update is
// dev_gepp's, so the factors are the same bit for bit.  Returns false at a zero pivot
// (pv[k] written for that column), like dev_gepp.
template <class T>
__device__ inline bool wave_gepp(int m, T *a, int *pv, int lane) {
    for (int k = 0; k < m; ++k) {
        const T akk = fabs(a[k * m + k]);
        // largest modulus below the diagonal, the first row on ties (NaN as -1)
        T vv = T(-1);
        int rr = m;
        if (lane > k && lane < m) {
            const T x = fabs(a[lane * m + k]);
            vv = x != x ? T(-1) : x;
            rr = lane;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const T ov = __shfl_xor(vv, off, 64);
            const int orr = __shfl_xor(rr, off, 64);
            if (ov > vv || (ov == vv && orr < rr)) {
                vv = ov;
                rr = orr;
            }
        }
        const int pr = (akk == akk && vv > akk) ? rr : k;
        const T amax = pr == k ? akk : vv;
        if (lane == 0) pv[k] = pr;
        if (amax == T(0)) {
            return false;
        }
        if (pr != k && lane < m) {
            const T t = a[k * m + lane];
            a[k * m + lane] = a[pr * m + lane];
            a[pr * m + lane] = t;
        }
        wave_sync();
        if (lane > k && lane < m) a[lane * m + k] = a[lane * m + k] / a[k * m + k];
        wave_sync();
        const int rest = m - k - 1;
        for (int e = lane; e < rest * rest; e += 64) {
            const int r = k + 1 + e / rest, c = k + 1 + e % rest;
            a[r * m + c] = a[r * m + c] - a[r * m + k] * a[k * m + c];
        }
        wave_sync();
    }
    return true;
}
// Smallest over largest pivot magnitude of a factored m x m block: a cheap stand-in for
// the reciprocal of its condition number (1 for a perfectly balanced block).
template <class T>
__device__ inline double dev_pivot_ratio(int m, const T *lu) {
    double mn = 0.0, mx = 0.0;
    for (int k = 0; k < m; ++k) {
        const double a = fabs((double)lu[k * m + k]);
        mn = k == 0 || a < mn ? a : mn;
        mx = a > mx ? a : mx;
    }
    return mx > 0.0 ? mn / mx : 0.0;
}
// Counts a factored pivot block whose pivot ratio is below `min_ratio` in err[3].
template <class T>
__device__ inline void dev_count_illcond(int m, const T *lu, double min_ratio, int *err) {
    if (min_ratio > 0.0 && dev_pivot_ratio<T>(m, lu) < min_ratio) atomicAdd(&err[3], 1);
}

// x <- L^{-1} P x
template <class T, class V>
__device__ inline void dev_lu_fwd(int m, const T *lu, const int *piv, V *x) {
    for (int k = 0; k < m; ++k) {
        int pk = piv[k];
        if (pk != k) { V t = x[k]; x[k] = x[pk]; x[pk] = t; }
    }
    for (int r = 0; r < m; ++r) {
        V s = x[r];
        for (int q = 0; q < r; ++q) s = s - V(lu[r * m + q]) * x[q];
        x[r] = s;
    }
}
// x <- U^{-1} x
template <class T, class V>
__device__ inline void dev_lu_bwd(int m, const T *lu, V *x) {
    for (int r = m - 1; r >= 0; --r) {
        V s = x[r];
        for (int q = r + 1; q < m; ++q) s = s - V(lu[r * m + q]) * x[q];
        x[r] = s / V(lu[r * m + r]);
    }
}
// Register versions for vectors of up to MAXM entries: the loops are unrolled to MAXM with
// guards, so the vector never leaves registers; operations and order are those above.
// x <- L^{-1} x (unit lower triangle; the row exchanges are applied beforehand)
template <class T, class V, int MAXM>
__device__ inline void reg_l_fwd(int m, const T *lu, V (&x)[MAXM]) {
#pragma unroll
    for (int r = 0; r < MAXM; ++r) {
        if (r < m) {
            V s = x[r];
#pragma unroll
            for (int q = 0; q < r; ++q) s = s - V(lu[r * m + q]) * x[q];
            x[r] = s;
        }
    }
}
// x <- U^{-1} x
template <class T, class V, int MAXM>
__device__ inline void reg_lu_bwd(int m, const T *lu, V (&x)[MAXM]) {
#pragma unroll
    for (int r = MAXM - 1; r >= 0; --r) {
        if (r < m) {
            V s = x[r];
#pragma unroll
            for (int q = r + 1; q < MAXM; ++q)
                if (q < m) s = s - V(lu[r * m + q]) * x[q];
            x[r] = s / V(lu[r * m + r]);
        }
    }
}
// row vector e <- e U^{-1}, e strided by `st`
template <class T>
__device__ inline void dev_row_solve_u(int m, const T *lu, T *e, int st) {
    for (int c = 0; c < m; ++c) {
        T s = e[c * st];
        for (int q = 0; q < c; ++q) s = s - e[q * st] * lu[q * m + c];
        e[c * st] = s / lu[c * m + c];
    }
}
// row vector e <- e L^{-1} P
template <class T>
__device__ inline void dev_row_solve_lp(int m, const T *lu, const int *piv, T *e, int st) {
    for (int c = m - 1; c >= 0; --c) {
        T s = e[c * st];
        for (int q = c + 1; q < m; ++q) s = s - e[q * st] * lu[q * m + c];
        e[c * st] = s;
    }
    for (int k = m - 1; k >= 0; --k) {
        int pk = piv[k];
        if (pk != k) { T t = e[k * st]; e[k * st] = e[pk * st]; e[pk * st] = t; }
    }
}
// drop rule: ||B||_F / (m n) < t, B given row-major with row stride `ld`
template <class T>
__device__ inline bool dev_drop(int m, int n, const T *b, int64_t ld, double t) {
    T s = T(0);
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < n; ++c) {
            T v = b[r * ld + c];
            s = s + v * v;
        }
    T thr = T(t) * T(m * n);
    return s < thr * thr;
}

// ---------------------------------------------------------------------------------
// Utilities (util.hip)
// ---------------------------------------------------------------------------------
// out[i] = sum_{j<i} in[j] for i in [0, n]; out has n+1 entries; returns the total.
int64_t scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, bool want_total = true);
int64_t scan_i32_to_i64(const int *in, int64_t *out, int64_t n, hipStream_t s, bool want_total = true);
int scan_i32(const int *in, int *out, int64_t n, hipStream_t s, bool want_total = true);
void fill_i32(int *p, int v, int64_t n, hipStream_t s);
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);
template <class T> void fill_val(T *p, T v, int64_t n, hipStream_t s);
void iota_i32(int *p, int64_t n, hipStream_t s);
// rowblk[r] = block of scalar row r from offsets rb[p+1]
void fill_rowblk(const int *rb, int p, int *rowblk, hipStream_t s);
int max_block_size(const int *rb, int p, hipStream_t s);

// Panel construction helpers (panel.hip)
// From ci/rp (+ column block offsets cb) compute co, wp, vp, sc and totals; rb/cb/rp/ci set.
template <class T> void panel_finish_layout(Panel<T> &a, hipStream_t s);
template <class T> void panel_set_blocks(Panel<T> &a, const std::vector<int> &rb, const std::vector<int> &cb, hipStream_t s);

// Compaction: dst takes the blocks with keep[k] != 0 of src rows selected by src_row_of[r]
// (dst row r <- src row src_row_of[r]), renaming block columns through newcol[src col].
// `vals` (may be NULL) overrides src.v as the source of the values.
template <class T>
void panel_compact(const Panel<T> &src, const T *vals, const int *keep, const int *src_row_of, int dst_p,
                   const int *newcol, const std::vector<int> &dst_rb, const std::vector<int> &dst_cb,
                   Panel<T> &dst, hipStream_t s);

// Host copy of a panel in the exported block-sparse-row format.
template <class T>
void panel_export(const Panel<T> &a, std::vector<int64_t> &rowptr, std::vector<int> &colidx,
                  std::vector<double> &vals, hipStream_t s);

// SpMV y = A x on the panel (spmv.hip); x indexed by sc, y by scalar row.
template <class T>
void panel_spmv(const Panel<T> &a, const double *x, double *y, hipStream_t s, int nv = 1);
template <class T>
double panel_spmv_bytes(const Panel<T> &a, bool with_b);
template <class T>
int autotune_spmv(Panel<T> &a, hipStream_t s);

}  // namespace vb
