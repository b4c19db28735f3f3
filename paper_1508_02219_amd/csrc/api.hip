// C ABI of the VBARMS library (declared in include/vbarms.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "factor.h"

using namespace vb;

struct vbarms_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    std::string last_error;
    int n = 0;
    int64_t nnz = 0;
    DBuf<int> perm;             // new position -> original row
    std::vector<int> bptr;      // host block offsets
    Panel<double> A;            // compressed matrix P_B A P_B^T
    bool have_A = false;
    int precision = VBARMS_F64;
    std::unique_ptr<Factors<double>> f64;
    std::unique_ptr<Factors<float>> f32;
    bool have_factors = false;
    DevErr err;
    int err_level = -1, err_block = -1;
    vbarms_fstats stats{};
    DBuf<double> wx, wy;        // permuted in/out vectors
    KrylovWork kw;
    KTimer kt;                  // optional kernel timing
    IlutHint ilut_hint;         // room the last-level ILUT needed so far
    bool graphs = true;         // replay the last-level sweeps from a captured graph
    vbarms_fparams params{};    // parameters of the last factorization
    // FP32 safeguards: redo in FP64 when a pivot block's pivot ratio is below min_pivot_ratio
    // (at factorization) or when FGMRES has not converged after f32_iter_limit steps
    bool fb_enable = true;
    int fb_iter_limit = 100;
    double fb_min_ratio = 1e-4;
};

namespace {

// Fixed device array for vbarms_spmv_noalloc: the permuted input and output vectors of one
// product (2 * VBARMS_NOALLOC_MAX_N doubles, 32 MiB), one copy per GPU the library runs on,
// held until the process ends.  Host code never uses the array's name as an address: its
// device address is read once per device (noalloc_scratch_init) and kept below.
__device__ __align__(256) double scratch[2 * (size_t)VBARMS_NOALLOC_MAX_N];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Reads the address of `scratch` on the current device (which must be `dev`) once.
void noalloc_scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(VBARMS_ERR_ARG, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev]) return;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        fail(VBARMS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = (double *)ptr;
}

double *noalloc_scratch(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr;
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit Timer(hipStream_t s_) : s(s_) {
        VB_HIP(hipEventCreate(&a));
        VB_HIP(hipEventCreate(&b));
        VB_HIP(hipEventRecord(a, s));
    }
    double stop() {
        VB_HIP(hipEventRecord(b, s));
        VB_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        VB_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct TimerScope {
    KTimer *prev;
    explicit TimerScope(KTimer *t) : prev(cur_ktimer()) { cur_ktimer() = t; }
    ~TimerScope() { cur_ktimer() = prev; }
};

template <class F>
int guarded(vbarms_t h, F &&body) {
    if (!h) return VBARMS_ERR_ARG;
    StreamScope scope(h->stream);  // device buffers are allocated and freed on the handle's stream
    TimerScope tscope(&h->kt);
    try {
        h->last_error.clear();
        VB_HIP(hipSetDevice(h->device));
        int rc = body();
        if (!h->kt.pend.empty()) {
            VB_HIP(hipStreamSynchronize(h->stream));
            h->kt.resolve();
        }
        return rc;
    } catch (const VbError &e) {
        h->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        h->last_error = "host allocation failed";
        return VBARMS_ERR_OOM;
    } catch (...) {
        h->last_error = "unexpected internal error";
        return VBARMS_ERR_HIP;
    }
}

// converts a device error record into an exception; returns the record's count of
// ill-conditioned pivot blocks
int check_dev_err(vbarms_t h, const char *stage) {
    std::vector<int> rec;
    to_host(rec, h->err.rec.p, 4, h->stream);
    if (rec[0] == 0) return rec[3];
    h->err_level = rec[1];
    h->err_block = rec[2];
    std::string msg = std::string(stage) + ": ";
    switch (rec[0]) {
    case VBARMS_ERR_SINGULAR:
        msg += "singular pivot block " + std::to_string(rec[2]) + " at level " + std::to_string(rec[1]);
        break;
    case VBARMS_ERR_NAN: msg += "NaN or Inf in the matrix (row " + std::to_string(rec[1]) + ")"; break;
    case VBARMS_ERR_OOM: msg += "capacity exceeded (level " + std::to_string(rec[1]) + ", row " + std::to_string(rec[2]) + ")"; break;
    default: msg += "inconsistent factor data (level " + std::to_string(rec[1]) + ", row " + std::to_string(rec[2]) + ")"; break;
    }
    fail(rec[0], msg);
    return rec[3];
}

void validate_csr(const vbarms_csr *A) {
    if (!A || A->n < 0 || A->nnz < 0) fail(VBARMS_ERR_ARG, "invalid CSR descriptor");
    if (A->n > 0 && (!A->rowptr || (A->nnz > 0 && (!A->col || !A->val))))
        fail(VBARMS_ERR_ARG, "NULL CSR array");
}

void finish_partition(vbarms_t h, const vbarms_csr *A, vbarms_cstats *st) {
    hipStream_t s = h->stream;
    h->err.reset(s);
    h->A = Panel<double>();
    panel_from_csr(A->n, A->rowptr, A->col, A->val, h->perm.p, h->bptr, h->A, h->err.rec.p, s);
    check_dev_err(h, "compress");
    h->stats.spmv_lanes = autotune_spmv<double>(h->A, s);
    h->have_A = true;
    h->have_factors = false;
    h->f64.reset();
    h->f32.reset();
    int maxb = 0;
    for (size_t i = 0; i + 1 < h->bptr.size(); ++i) maxb = std::max(maxb, h->bptr[i + 1] - h->bptr[i]);
    if (st) {
        st->nblocks = (int)h->bptr.size() - 1;
        st->max_block = maxb;
        st->nnz_blocks = h->A.nb;
        st->av_bd = h->A.nv > 0 ? (double)A->nnz / (double)h->A.nv : 1.0;
        st->av_bs = st->nblocks > 0 ? (double)A->n / st->nblocks : 0.0;
    }
    h->wx.alloc(std::max(A->n, 1));
    h->wy.alloc(std::max(A->n, 1));
}

// Factors the compressed matrix in precision T; returns the number of pivot blocks whose
// pivot ratio fell below the handle's threshold.
template <class T>
int factor_impl(vbarms_t h, const vbarms_fparams *p, std::unique_ptr<Factors<T>> &fp) {
    hipStream_t s = h->stream;
    fp.reset(new Factors<T>());
    Factors<T> &f = *fp;
    const int levels = p->levels;
    f.lev.reserve(levels + 1);
    int ill_levels = 0;
    Panel<T> cur;
    panel_convert<double, T>(h->A, cur, s);
    h->err.reset(s);
    for (int l = 0; l < levels; ++l) {
        if (cur.p == 0) break;
        Timer tm(s);
        f.lev.emplace_back();
        Panel<T> next;
        factor_level<T>(f.lev[l], std::move(cur), l, p->droptol[l], p->drop_schur, p->is_order, p->group_rows,
                        h->fb_min_ratio, next, h->err.rec.p, s);
        f.nlev = l + 1;
        ill_levels = check_dev_err(h, "factor");
        f.level_ms[l] = tm.stop();
        cur = std::move(next);
        if (f.lev[l].nis == 0) break;
    }
    f.last.A = std::move(cur);
    f.last.use_graph = h->graphs;
    Timer tm(s);
    factor_last<T>(f.last, p->droptol[levels], h->fb_min_ratio, f.nlev, h->ilut_hint, h->err.rec.p, s);
    const int ill = ill_levels + check_dev_err(h, "last-level ILUT");
    f.ilut_ms = tm.stop();
    h->stats.levels = f.nlev;
    h->stats.last_p = f.last.A.p;
    for (int l = 0; l < VBARMS_MAX_LEVELS; ++l) h->stats.factor_level_ms[l] = l < f.nlev ? f.level_ms[l] : 0.0;
    h->stats.ilut_ms = f.ilut_ms;
    h->stats.ilut_waves = f.last.waves;
    h->stats.ilut_attempts = f.last.attempts;
    int64_t vals = 0;
    // bytes of one application: per level the pivot-block factors, G, W and their column
    // lists, the pivots and about six passes over the level's vectors; then both sweeps
    double abytes = f.last.sweep_bytes;
    for (int l = 0; l < f.nlev; ++l) {
        const Level<T> &L = f.lev[l];
        std::vector<int64_t> d;
        to_host(d, L.dlu_off.p + L.nis, 1, s);
        vals += d[0] + L.G.nv + L.W.nv;
        abytes += (double)sizeof(T) * (double)(d[0] + L.G.nv + L.W.nv) + 4.0 * (double)(L.G.nw + L.W.nw) +
                  4.0 * L.n_is + 4.0 * L.n + 8.0 * 6.0 * L.n;
    }
    f.apply_bytes = abytes;
    {
        std::vector<int64_t> d;
        to_host(d, f.last.dl_off.p + f.last.A.p, 1, s);
        vals += d[0] + f.last.L.nv + f.last.U.nv;
        const LastLevel<T> &ll = f.last;
        const int64_t nlast = ll.A.h_rb.empty() ? 0 : ll.A.h_rb.back();
        h->stats.ilut_result_bytes = (double)sizeof(T) * (double)(ll.A.nv + ll.L.nv + ll.U.nv + d[0]) +
                                     4.0 * (double)(ll.A.nb + ll.L.nb + ll.U.nb) + 4.0 * (double)nlast;
    }
    h->stats.factor_values = vals;
    return ill;
}

// Replaces FP32 factors by FP64 factors of the same matrix and parameters.
void refactor_fp64(vbarms_t h) {
    vbarms_fparams q = h->params;
    q.precision = VBARMS_F64;
    h->have_factors = false;
    h->f32.reset();
    h->precision = VBARMS_F64;
    h->stats.illcond_blocks = factor_impl<double>(h, &q, h->f64);
    h->have_factors = true;
}

// M^{-1} in the compressed numbering
// y = M^{-1} x for nv vectors (n apart), in the compressed numbering
void precond_apply(vbarms_t h, const double *x, double *y, int nv = 1) {
    if (h->precision == VBARMS_F32) {
        KScope ks(VBARMS_K_APPLY, h->f32->apply_bytes * nv, h->stream);
        solve_levels<float>(*h->f32, 0, x, y, nv, h->err.rec.p, h->stream);
    } else {
        KScope ks(VBARMS_K_APPLY, h->f64->apply_bytes * nv, h->stream);
        solve_levels<double>(*h->f64, 0, x, y, nv, h->err.rec.p, h->stream);
    }
}

template <class T>
int export_level_matrix(vbarms_t h, Factors<T> &f, int which, int level, int64_t *dims, int32_t *rb, int32_t *cb,
                        int64_t *rowptr, int32_t *colidx, double *vals, int32_t *piv) {
    hipStream_t s = h->stream;
    const Panel<T> *P = nullptr;
    if (which == VBARMS_M_LAST) P = &f.last.A;
    else if (which == VBARMS_M_L) P = &f.last.L;
    else if (which == VBARMS_M_U) P = &f.last.U;
    else if (which == VBARMS_M_DL) {
        int p = f.last.A.p;
        std::vector<int64_t> off;
        to_host(off, f.last.dl_off.p, p + 1, s);
        if (dims) { dims[0] = p; dims[1] = p; dims[2] = p; dims[3] = off[p]; return VBARMS_OK; }
        for (int i = 0; i <= p; ++i) { rb[i] = f.last.A.h_rb[i]; cb[i] = f.last.A.h_rb[i]; rowptr[i] = i; }
        for (int i = 0; i < p; ++i) colidx[i] = i;
        std::vector<T> v;
        to_host(v, f.last.dl.p, off[p], s);
        for (int64_t k = 0; k < off[p]; ++k) vals[k] = (double)v[k];
        if (piv) {
            std::vector<int> pv;
            to_host(pv, f.last.dl_piv.p, f.last.A.h_rb[p], s);
            std::copy(pv.begin(), pv.end(), piv);
        }
        return VBARMS_OK;
    } else {
        if (level < 0 || level >= f.nlev) fail(VBARMS_ERR_ARG, "level out of range");
        Level<T> &L = f.lev[level];
        if (which == VBARMS_M_A) P = &L.A;
        else if (which == VBARMS_M_AS) P = &L.As;
        else if (which == VBARMS_M_G) P = &L.G;
        else if (which == VBARMS_M_W) P = &L.W;
        else if (which == VBARMS_M_D) {
            int nis = L.nis;
            std::vector<int64_t> off;
            to_host(off, L.dlu_off.p, nis + 1, s);
            if (dims) { dims[0] = nis; dims[1] = nis; dims[2] = nis; dims[3] = off[nis]; return VBARMS_OK; }
            for (int i = 0; i <= nis; ++i) { rb[i] = L.h_is_rb[i]; cb[i] = L.h_is_rb[i]; rowptr[i] = i; }
            for (int i = 0; i < nis; ++i) colidx[i] = i;
            std::vector<T> v;
            to_host(v, L.dlu.p, off[nis], s);
            for (int64_t k = 0; k < off[nis]; ++k) vals[k] = (double)v[k];
            if (piv) {
                std::vector<int> pv;
                to_host(pv, L.dpiv.p, L.n_is, s);
                std::copy(pv.begin(), pv.end(), piv);
            }
            return VBARMS_OK;
        } else {
            fail(VBARMS_ERR_ARG, "unknown matrix selector");
        }
    }
    if (dims) {
        dims[0] = P->p;
        dims[1] = P->q;
        dims[2] = P->nb;
        dims[3] = P->nv;
        return VBARMS_OK;
    }
    std::copy(P->h_rb.begin(), P->h_rb.end(), rb);
    std::copy(P->h_cb.begin(), P->h_cb.end(), cb);
    std::vector<int64_t> rp;
    std::vector<int> ci;
    std::vector<double> v;
    panel_export<T>(*P, rp, ci, v, s);
    std::copy(rp.begin(), rp.end(), rowptr);
    std::copy(ci.begin(), ci.end(), colidx);
    std::copy(v.begin(), v.end(), vals);
    return VBARMS_OK;
}

template <class T>
Level<T> &level_of(Factors<T> &f, int level) {
    if (level < 0 || level >= f.nlev) fail(VBARMS_ERR_ARG, "level out of range");
    return f.lev[level];
}

void need_factors(vbarms_t h) {
    if (!h->have_factors) fail(VBARMS_ERR_STATE, "no factorization: call vbarms_factor first");
}

}  // namespace

// Several independent systems held as one block-diagonal system (vbarms_batch_*).
struct vbarms_batch_ctx {
    vbarms_t h = nullptr;          // handle of the combined system
    std::vector<int64_t> off;      // first row of every system in the combined numbering
    Segments seg;                  // the systems of one vector
    Segments segv;                 // the systems of seg_nv vectors one after another
    int seg_nv = 0;
    BatchKrylovWork kw;
    std::string last_error;
    bool have_factors = false;
};

namespace {

// rows [off_s, off_s + n_s) of the combined CSR from system s: column indices shifted by
// off_s, row offsets by the entries of the systems before it
__global__ void k_batch_rows(int n, const int64_t *rp, int64_t row0, int64_t nnz0, int64_t *crp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) crp[row0 + i] = nnz0 + rp[i];
}
__global__ void k_batch_cols(int64_t nnz, const int *ci, int col0, int *cci) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) cci[k] = ci[k] + col0;
}

template <class F>
int batch_guarded(vbarms_batch_t b, F &&body) {
    if (!b) return VBARMS_ERR_ARG;
    StreamScope scope(b->h->stream);
    try {
        b->last_error.clear();
        VB_HIP(hipSetDevice(b->h->device));
        return body();
    } catch (const VbError &e) {
        b->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        b->last_error = "host allocation failed";
        return VBARMS_ERR_OOM;
    } catch (...) {
        b->last_error = "unexpected internal error";
        return VBARMS_ERR_HIP;
    }
}

}  // namespace

extern "C" {

int vbarms_create(vbarms_t *out, void *hip_stream) {
    if (!out) return VBARMS_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return VBARMS_ERR_HIP;
    vbarms_ctx *h = new (std::nothrow) vbarms_ctx();
    if (!h) return VBARMS_ERR_OOM;
    if (hipGetDevice(&h->device) != hipSuccess) { delete h; return VBARMS_ERR_HIP; }
    h->stream = (hipStream_t)hip_stream;
    int rc = guarded(h, [&] {
        h->err.reset(h->stream);
        noalloc_scratch_init(h->device);
        return VBARMS_OK;
    });
    if (rc != VBARMS_OK) { delete h; return rc; }
    *out = h;
    return VBARMS_OK;
}

int vbarms_destroy(vbarms_t h) {
    if (!h) return VBARMS_ERR_ARG;
    (void)hipSetDevice(h->device);
    hipStream_t s = h->stream;
    {
        StreamScope scope(s);  // buffers are released in stream order
        delete h;
    }
    (void)hipStreamSynchronize(s);
    return VBARMS_OK;
}

const char *vbarms_last_error(vbarms_t h) { return h ? h->last_error.c_str() : "invalid handle"; }

int vbarms_compress(vbarms_t h, const vbarms_csr *A, double tau, int32_t *perm, int32_t *bptr, vbarms_cstats *st) {
    return guarded(h, [&] {
        validate_csr(A);
        if (!(tau > 0.0 && tau <= 1.0)) fail(VBARMS_ERR_ARG, "tau must lie in (0, 1]");
        hipStream_t s = h->stream;
        Timer tm(s);
        h->n = A->n;
        h->nnz = A->nnz;
        h->perm.alloc(std::max(A->n, 1));
        h->bptr = compress_gpu(A->n, A->rowptr, A->col, tau, h->perm.p, s);
        finish_partition(h, A, st);
        if (perm && A->n) VB_HIP(hipMemcpyAsync(perm, h->perm.p, sizeof(int) * A->n, hipMemcpyDeviceToDevice, s));
        if (bptr) to_device(bptr, h->bptr.data(), h->bptr.size(), s);
        VB_HIP(hipStreamSynchronize(s));
        h->stats.compress_ms = tm.stop();
        h->stats.nnz = A->nnz;
        return VBARMS_OK;
    });
}

int vbarms_compress_graph(vbarms_t h, const vbarms_csr *A, double mu, int32_t *perm, int32_t *bptr,
                          vbarms_cstats *st) {
    return guarded(h, [&] {
        validate_csr(A);
        if (!(mu > 0.0 && mu <= 1.0)) fail(VBARMS_ERR_ARG, "mu must lie in (0, 1]");
        hipStream_t s = h->stream;
        Timer tm(s);
        h->n = A->n;
        h->nnz = A->nnz;
        std::vector<int64_t> rp;
        std::vector<int> ci;
        to_host(rp, A->rowptr, (size_t)A->n + 1, s);
        to_host(ci, A->col, (size_t)A->nnz, s);
        for (int64_t k = 0; k < A->nnz; ++k)
            if (ci[k] < 0 || ci[k] >= A->n) fail(VBARMS_ERR_ARG, "column index out of range");
        std::vector<int> hperm;
        h->bptr = graph_compress_host(A->n, rp, ci, mu, hperm);
        h->perm.alloc(std::max(A->n, 1));
        to_device(h->perm.p, hperm.data(), hperm.size(), s);
        finish_partition(h, A, st);
        if (perm && A->n) VB_HIP(hipMemcpyAsync(perm, h->perm.p, sizeof(int) * A->n, hipMemcpyDeviceToDevice, s));
        if (bptr) to_device(bptr, h->bptr.data(), h->bptr.size(), s);
        VB_HIP(hipStreamSynchronize(s));  // host vectors are copy sources
        h->stats.compress_ms = tm.stop();
        h->stats.nnz = A->nnz;
        return VBARMS_OK;
    });
}

int vbarms_set_partition(vbarms_t h, const vbarms_csr *A, const int32_t *perm, const int32_t *bptr, int32_t p,
                         vbarms_cstats *st) {
    return guarded(h, [&] {
        validate_csr(A);
        if (p < 0 || (A->n > 0 && (!perm || !bptr))) fail(VBARMS_ERR_ARG, "invalid partition");
        hipStream_t s = h->stream;
        h->n = A->n;
        h->nnz = A->nnz;
        h->perm.alloc(std::max(A->n, 1));
        if (A->n) VB_HIP(hipMemcpyAsync(h->perm.p, perm, sizeof(int) * A->n, hipMemcpyDeviceToDevice, s));
        to_host(h->bptr, bptr, p + 1, s);
        if (h->bptr[0] != 0 || h->bptr[p] != A->n) fail(VBARMS_ERR_ARG, "bptr must run from 0 to n");
        for (int i = 0; i < p; ++i)
            if (h->bptr[i + 1] <= h->bptr[i]) fail(VBARMS_ERR_ARG, "empty or decreasing block in bptr");
        finish_partition(h, A, st);
        h->stats.nnz = A->nnz;
        return VBARMS_OK;
    });
}

int vbarms_factor(vbarms_t h, const vbarms_fparams *p) {
    return guarded(h, [&] {
        if (!p || p->levels < 0 || p->levels > VBARMS_MAX_LEVELS) fail(VBARMS_ERR_ARG, "invalid factor parameters");
        for (int l = 0; l <= p->levels; ++l)
            if (!(p->droptol[l] >= 0.0) || !std::isfinite(p->droptol[l])) fail(VBARMS_ERR_ARG, "invalid drop tolerance");
        if (p->precision != VBARMS_F64 && p->precision != VBARMS_F32) fail(VBARMS_ERR_ARG, "invalid precision");
        if (p->is_order != VBARMS_IS_NATURAL && p->is_order != VBARMS_IS_WEIGHTED)
            fail(VBARMS_ERR_ARG, "invalid independent-set order");
        if (p->group_rows < 0 || p->group_rows > VBARMS_MAX_BLOCK) fail(VBARMS_ERR_ARG, "invalid group_rows");
        if (!h->have_A) fail(VBARMS_ERR_STATE, "no compressed matrix: call vbarms_compress first");
        h->have_factors = false;
        h->err_level = h->err_block = -1;
        h->f64.reset();
        h->f32.reset();
        h->precision = p->precision;
        h->params = *p;
        h->stats.fp64_fallback = 0;
        Timer tm(h->stream);
        if (p->precision == VBARMS_F32) {
            bool redo = false;
            try {
                h->stats.illcond_blocks = factor_impl<float>(h, p, h->f32);
                redo = h->fb_enable && h->stats.illcond_blocks > 0;
            } catch (const VbError &e) {
                // a pivot block that is singular in FP32 may not be in FP64
                if (!h->fb_enable || e.code != VBARMS_ERR_SINGULAR) throw;
                h->stats.illcond_blocks = 1;
                redo = true;
            }
            if (redo) {
                // an FP32 pivot block is ill-conditioned: the whole factorization runs in FP64
                h->err_level = h->err_block = -1;
                refactor_fp64(h);
                h->stats.fp64_fallback = 1;
            }
        } else {
            h->stats.illcond_blocks = factor_impl<double>(h, p, h->f64);
        }
        h->stats.factor_ms = tm.stop();
        h->have_factors = true;
        return VBARMS_OK;
    });
}

int vbarms_error_location(vbarms_t h, int32_t *level, int32_t *block) {
    if (!h) return VBARMS_ERR_ARG;
    if (level) *level = h->err_level;
    if (block) *block = h->err_block;
    return VBARMS_OK;
}

int vbarms_apply(vbarms_t h, const double *x, double *y) {
    return guarded(h, [&] {
        need_factors(h);
        if (h->n > 0 && (!x || !y)) fail(VBARMS_ERR_ARG, "NULL vector");
        hipStream_t s = h->stream;
        h->err.reset(s);
        gather_perm(h->n, h->perm.p, x, h->wx.p, s);
        precond_apply(h, h->wx.p, h->wy.p);
        scatter_perm(h->n, h->perm.p, h->wy.p, y, s);
        check_dev_err(h, "apply");
        return VBARMS_OK;
    });
}

int vbarms_spmv(vbarms_t h, const double *x, double *y) {
    return guarded(h, [&] {
        if (!h->have_A) fail(VBARMS_ERR_STATE, "no compressed matrix");
        if (h->n > 0 && (!x || !y)) fail(VBARMS_ERR_ARG, "NULL vector");
        hipStream_t s = h->stream;
        gather_perm(h->n, h->perm.p, x, h->wx.p, s);
        panel_spmv<double>(h->A, h->wx.p, h->wy.p, s);
        scatter_perm(h->n, h->perm.p, h->wy.p, y, s);
        return VBARMS_OK;
    });
}

int vbarms_set_spmv_lanes(vbarms_t h, int32_t lanes) {
    return guarded(h, [&] {
        if (!h->have_A) fail(VBARMS_ERR_STATE, "no compressed matrix");
        if (lanes != 4 && lanes != 8 && lanes != 16 && lanes != 32)
            fail(VBARMS_ERR_ARG, "lanes must be 4, 8, 16 or 32");
        h->A.tg = lanes;
        h->stats.spmv_lanes = lanes;
        return VBARMS_OK;
    });
}

int vbarms_spmv_noalloc(vbarms_t h, const double *x, double *y) {
    return guarded(h, [&] {
        if (!h->have_A) fail(VBARMS_ERR_STATE, "no compressed matrix");
        if (h->n > 0 && (!x || !y)) fail(VBARMS_ERR_ARG, "NULL vector");
        if ((int64_t)h->n > (int64_t)VBARMS_NOALLOC_MAX_N)
            fail(VBARMS_ERR_ARG, "n = " + std::to_string(h->n) + " exceeds VBARMS_NOALLOC_MAX_N = " +
                                     std::to_string((int64_t)VBARMS_NOALLOC_MAX_N));
        double *sx = noalloc_scratch(h->device);
        if (!sx) fail(VBARMS_ERR_STATE, "no scratch address for this device");
        double *sy = sx + (size_t)VBARMS_NOALLOC_MAX_N;
        hipStream_t s = h->stream;
        gather_perm(h->n, h->perm.p, x, sx, s);
        panel_spmv<double>(h->A, sx, sy, s);
        scatter_perm(h->n, h->perm.p, sy, y, s);
        return VBARMS_OK;
    });
}

int vbarms_solve(vbarms_t h, const double *b, double *x, double tol, int32_t restart, int32_t maxit,
                 vbarms_sinfo *info) {
    return guarded(h, [&] {
        need_factors(h);
        if (restart < 1 || maxit < 0 || !(tol >= 0.0)) fail(VBARMS_ERR_ARG, "invalid solver parameters");
        if (h->n > 0 && (!x || !b)) fail(VBARMS_ERR_ARG, "NULL vector");
        hipStream_t s = h->stream;
        Timer tm(s);
        h->err.reset(s);
        DBuf<double> bc(std::max(h->n, 1)), xc(std::max(h->n, 1));
        gather_perm(h->n, h->perm.p, b, bc.p, s);
        gather_perm(h->n, h->perm.p, x, xc.p, s);
        auto pre = [&](const double *in, double *out) { precond_apply(h, in, out); };
        vbarms_sinfo i1{}, i2{};
        int st;
        if (h->precision == VBARMS_F32 && h->fb_enable && h->fb_iter_limit < maxit) {
            // FP32 factors get fb_iter_limit Arnoldi steps; if FGMRES has not converged by
            // then, the factors are recomputed in FP64 and FGMRES continues from its iterate
            st = fgmres_run(h->A, h->kw, bc.p, xc.p, tol, restart, h->fb_iter_limit, pre, &i1, s);
            check_dev_err(h, "solve");
            if (st == VBARMS_NOT_CONVERGED) {
                refactor_fp64(h);
                h->stats.fp64_fallback = 2;
                h->err.reset(s);
                st = fgmres_run(h->A, h->kw, bc.p, xc.p, tol, restart, maxit - i1.iters, pre, &i2, s);
                i2.iters += i1.iters;
                i2.restarts += i1.restarts;
                i2.fp64_refactor = 1;
                i1 = i2;
            }
        } else {
            st = fgmres_run(h->A, h->kw, bc.p, xc.p, tol, restart, maxit, pre, &i1, s);
        }
        if (info) *info = i1;
        check_dev_err(h, "solve");
        scatter_perm(h->n, h->perm.p, xc.p, x, s);
        VB_HIP(hipStreamSynchronize(s));
        h->stats.solve_ms = tm.stop();
        return st;
    });
}

int vbarms_device_memory(int64_t *out) {
    if (!out) return VBARMS_ERR_ARG;
    const DevCacheStats c = dev_cache_stats();
    out[0] = (int64_t)c.live_bytes;
    out[1] = (int64_t)c.cached_bytes;
    out[2] = (int64_t)c.peak_bytes;
    out[3] = c.runtime_allocs;
    return VBARMS_OK;
}

int vbarms_set_fp64_fallback(vbarms_t h, int32_t enable, int32_t f32_iter_limit, double min_pivot_ratio) {
    return guarded(h, [&] {
        if (f32_iter_limit < 0 || !(min_pivot_ratio >= 0.0) || !(min_pivot_ratio <= 1.0))
            fail(VBARMS_ERR_ARG, "invalid fallback settings");
        h->fb_enable = enable != 0;
        h->fb_iter_limit = f32_iter_limit;
        h->fb_min_ratio = min_pivot_ratio;
        return VBARMS_OK;
    });
}

int vbarms_batch_create(vbarms_batch_t *out, void *hip_stream) {
    if (!out) return VBARMS_ERR_ARG;
    *out = nullptr;
    vbarms_batch_ctx *b = new (std::nothrow) vbarms_batch_ctx();
    if (!b) return VBARMS_ERR_OOM;
    int rc = vbarms_create(&b->h, hip_stream);
    if (rc != VBARMS_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return VBARMS_OK;
}

int vbarms_batch_destroy(vbarms_batch_t b) {
    if (!b) return VBARMS_ERR_ARG;
    vbarms_t h = b->h;
    {
        StreamScope scope(h->stream);  // buffers are released in stream order
        (void)hipSetDevice(h->device);
        b->seg = Segments();
        b->segv = Segments();
        b->seg_nv = 0;
        b->kw = BatchKrylovWork();
    }
    delete b;
    return vbarms_destroy(h);
}

const char *vbarms_batch_last_error(vbarms_batch_t b) { return b ? b->last_error.c_str() : "invalid handle"; }

vbarms_t vbarms_batch_handle(vbarms_batch_t b) { return b ? b->h : nullptr; }

int vbarms_batch_factor(vbarms_batch_t b, int32_t nsys, const vbarms_csr *systems, double tau,
                        const vbarms_fparams *p) {
    return batch_guarded(b, [&] {
        if (nsys < 1 || !systems || !p) fail(VBARMS_ERR_ARG, "invalid batch");
        vbarms_t h = b->h;
        hipStream_t s = h->stream;
        b->have_factors = false;
        std::vector<int64_t> off(nsys + 1, 0), noff(nsys + 1, 0);
        for (int q = 0; q < nsys; ++q) {
            validate_csr(&systems[q]);
            off[q + 1] = off[q] + systems[q].n;
            noff[q + 1] = noff[q] + systems[q].nnz;
        }
        if (off[nsys] > INT32_MAX) fail(VBARMS_ERR_ARG, "the systems hold more than 2^31 - 1 rows together");
        const int ntot = (int)off[nsys];
        // the block-diagonal matrix of all systems, assembled on the device
        DBuf<int64_t> crp(ntot + 1);
        DBuf<int> cci(std::max<int64_t>(noff[nsys], 1));
        DBuf<double> cva(std::max<int64_t>(noff[nsys], 1));
        for (int q = 0; q < nsys; ++q) {
            const vbarms_csr &A = systems[q];
            if (A.n > 0) {
                k_batch_rows<<<grid_for(A.n, 256), 256, 0, s>>>(A.n, A.rowptr, off[q], noff[q], crp.p);
                VB_LAUNCH_CHECK();
            }
            if (A.nnz > 0) {
                k_batch_cols<<<grid_for(A.nnz, 256), 256, 0, s>>>(A.nnz, A.col, (int)off[q], cci.p + noff[q]);
                VB_LAUNCH_CHECK();
                VB_HIP(hipMemcpyAsync(cva.p + noff[q], A.val, sizeof(double) * A.nnz, hipMemcpyDeviceToDevice, s));
            }
        }
        to_device(crp.p + ntot, &noff[nsys], 1, s);
        VB_HIP(hipStreamSynchronize(s));  // noff is a copy source
        vbarms_csr C{ntot, noff[nsys], crp.p, cci.p, cva.p};
        int rc = vbarms_compress(h, &C, tau, nullptr, nullptr, nullptr);
        if (rc != VBARMS_OK) fail(rc, std::string("batch compress: ") + h->last_error);
        // Rows of different systems share no column, so no block spans two systems, and
        // blocks follow their smallest row: every system keeps its row range in the
        // compressed numbering.
        b->off = off;
        b->seg.build(off, s);
        b->seg_nv = 0;  // the multi-vector segments follow the new systems
        rc = vbarms_factor(h, p);
        if (rc != VBARMS_OK) fail(rc, std::string("batch factor: ") + h->last_error);
        b->have_factors = true;
        return VBARMS_OK;
    });
}

int vbarms_batch_offsets(vbarms_batch_t b, int64_t *off) {
    if (!b || !off) return VBARMS_ERR_ARG;
    std::copy(b->off.begin(), b->off.end(), off);
    return VBARMS_OK;
}

int vbarms_batch_solve(vbarms_batch_t b, const double *B, double *X, int32_t nrhs, double tol, int32_t restart,
                       int32_t maxit, vbarms_sinfo *info) {
    return batch_guarded(b, [&] {
        if (!b->have_factors) fail(VBARMS_ERR_STATE, "no factorization: call vbarms_batch_factor first");
        if (nrhs < 1 || restart < 1 || maxit < 0 || !(tol >= 0.0) || !B || !X)
            fail(VBARMS_ERR_ARG, "invalid solver parameters");
        vbarms_t h = b->h;
        hipStream_t s = h->stream;
        Timer tm(s);
        const int64_t n = b->off.back();
        const int ns = b->seg.nseg;
        // right-hand sides per lockstep run: the Krylov bases of a vector take
        // (2 restart + 1) n doubles; a run keeps them within a third of the device
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = (size_t)64 << 30;
        const double per_rhs = 8.0 * (2.0 * restart + 4.0) * (double)std::max<int64_t>(n, 1);
        const int wave = (int)std::max<double>(
            1.0, std::min<double>(std::min(nrhs, 1024), std::floor(tot / 3.0 / per_rhs)));
        DBuf<double> bc((size_t)std::max<int64_t>(n, 1) * wave), xc((size_t)std::max<int64_t>(n, 1) * wave);
        auto pre = [&](const double *in, double *out, int nv) { precond_apply(h, in, out, nv); };
        std::vector<vbarms_sinfo> inf;
        int worst = VBARMS_OK;
        for (int r0 = 0; r0 < nrhs; r0 += wave) {
            const int nv = std::min(wave, nrhs - r0);
            if (b->seg_nv != nv) {  // segments of nv copies of the combined numbering
                std::vector<int64_t> offv((size_t)nv * ns + 1);
                for (int r = 0; r < nv; ++r)
                    for (int q = 0; q < ns; ++q) offv[(size_t)r * ns + q] = (int64_t)r * n + b->off[q];
                offv[(size_t)nv * ns] = (int64_t)nv * n;
                b->segv.build(offv, s);
                b->seg_nv = nv;
            }
            h->err.reset(s);
            for (int r = 0; r < nv; ++r) {
                gather_perm((int)n, h->perm.p, B + (int64_t)(r0 + r) * n, bc.p + (int64_t)r * n, s);
                gather_perm((int)n, h->perm.p, X + (int64_t)(r0 + r) * n, xc.p + (int64_t)r * n, s);
            }
            const int st = fgmres_batch_run(h->A, nv, b->kw, b->segv, bc.p, xc.p, tol, restart, maxit, pre, inf, s);
            check_dev_err(h, "batch solve");
            for (int r = 0; r < nv; ++r)
                scatter_perm((int)n, h->perm.p, xc.p + (int64_t)r * n, X + (int64_t)(r0 + r) * n, s);
            if (st != VBARMS_OK) worst = VBARMS_NOT_CONVERGED;
            if (info)
                for (int r = 0; r < nv; ++r)
                    for (int q = 0; q < ns; ++q) info[(int64_t)(r0 + r) * ns + q] = inf[(size_t)r * ns + q];
        }
        VB_HIP(hipStreamSynchronize(s));
        h->stats.solve_ms = tm.stop();
        return worst;
    });
}

int vbarms_get_stats(vbarms_t h, vbarms_fstats *st) {
    if (!h || !st) return VBARMS_ERR_ARG;
    *st = h->stats;
    return VBARMS_OK;
}

int vbarms_features(vbarms_t h, const vbarms_csr *A, float *f) {
    return guarded(h, [&] {
        validate_csr(A);
        if (!f) fail(VBARMS_ERR_ARG, "NULL feature output");
        matrix_features(A->n, A->nnz, A->rowptr, A->col, A->val, f, h->stream);
        return VBARMS_OK;
    });
}

int vbarms_set_graphs(vbarms_t h, int32_t enable) {
    return guarded(h, [&] {
        h->graphs = enable != 0;
        if (h->f64) h->f64->last.use_graph = h->graphs;
        if (h->f32) h->f32->last.use_graph = h->graphs;
        return VBARMS_OK;
    });
}

int vbarms_set_timing(vbarms_t h, int32_t enable) {
    return guarded(h, [&] {
        VB_HIP(hipStreamSynchronize(h->stream));
        h->kt.reset();
        h->kt.on = enable != 0;
        return VBARMS_OK;
    });
}

int vbarms_kernel_stats(vbarms_t h, vbarms_kstat *out) {
    if (!out) return VBARMS_ERR_ARG;
    return guarded(h, [&] {
        VB_HIP(hipStreamSynchronize(h->stream));
        h->kt.resolve();
        for (int c = 0; c < VBARMS_K_COUNT; ++c) out[c] = h->kt.tot[c];
        return VBARMS_OK;
    });
}

int vbarms_num_levels(vbarms_t h, int32_t *levels) {
    return guarded(h, [&] {
        need_factors(h);
        *levels = h->precision == VBARMS_F32 ? h->f32->nlev : h->f64->nlev;
        return VBARMS_OK;
    });
}

int vbarms_level_info(vbarms_t h, int32_t level, int32_t *info) {
    return guarded(h, [&] {
        need_factors(h);
        auto fill = [&](auto &f) {
            auto &L = level_of(f, level);
            info[0] = L.p; info[1] = L.n; info[2] = L.nis; info[3] = L.n_is; info[4] = L.nis_sn;
        };
        if (h->precision == VBARMS_F32) fill(*h->f32); else fill(*h->f64);
        return VBARMS_OK;
    });
}

int vbarms_level_is(vbarms_t h, int32_t level, int32_t *is_list) {
    return guarded(h, [&] {
        need_factors(h);
        auto get = [&](auto &f) {
            auto &L = level_of(f, level);
            if (!L.h_gptr.empty()) {
                std::copy(L.h_members.begin(), L.h_members.end(), is_list);
                return;
            }
            std::vector<int> v;
            to_host(v, L.is_list.p, L.nis, h->stream);
            std::copy(v.begin(), v.end(), is_list);
        };
        if (h->precision == VBARMS_F32) get(*h->f32); else get(*h->f64);
        return VBARMS_OK;
    });
}

int vbarms_level_groups(vbarms_t h, int32_t level, int32_t *gptr) {
    return guarded(h, [&] {
        need_factors(h);
        auto get = [&](auto &f) {
            auto &L = level_of(f, level);
            if (!L.h_gptr.empty()) std::copy(L.h_gptr.begin(), L.h_gptr.end(), gptr);
            else
                for (int g = 0; g <= L.nis; ++g) gptr[g] = g;
        };
        if (h->precision == VBARMS_F32) get(*h->f32); else get(*h->f64);
        return VBARMS_OK;
    });
}

int vbarms_level_scaling(vbarms_t h, int32_t level, double *s1, double *s2) {
    return guarded(h, [&] {
        need_factors(h);
        auto get = [&](auto &f) {
            auto &L = level_of(f, level);
            std::vector<double> v;
            to_host(v, L.s1.p, L.n, h->stream);
            std::copy(v.begin(), v.end(), s1);
            to_host(v, L.s2.p, L.n, h->stream);
            std::copy(v.begin(), v.end(), s2);
        };
        if (h->precision == VBARMS_F32) get(*h->f32); else get(*h->f64);
        return VBARMS_OK;
    });
}

int vbarms_matrix_dims(vbarms_t h, int32_t which, int32_t level, int64_t *dims) {
    return guarded(h, [&] {
        need_factors(h);
        if (!dims) fail(VBARMS_ERR_ARG, "NULL dims");
        if (h->precision == VBARMS_F32)
            return export_level_matrix<float>(h, *h->f32, which, level, dims, nullptr, nullptr, nullptr, nullptr,
                                              nullptr, nullptr);
        return export_level_matrix<double>(h, *h->f64, which, level, dims, nullptr, nullptr, nullptr, nullptr, nullptr,
                                           nullptr);
    });
}

int vbarms_matrix_get(vbarms_t h, int32_t which, int32_t level, int32_t *rb, int32_t *cb, int64_t *rowptr,
                      int32_t *colidx, double *vals, int32_t *piv) {
    return guarded(h, [&] {
        need_factors(h);
        if (!rb || !cb || !rowptr || !colidx || !vals) fail(VBARMS_ERR_ARG, "NULL output array");
        if (h->precision == VBARMS_F32)
            return export_level_matrix<float>(h, *h->f32, which, level, nullptr, rb, cb, rowptr, colidx, vals, piv);
        return export_level_matrix<double>(h, *h->f64, which, level, nullptr, rb, cb, rowptr, colidx, vals, piv);
    });
}

}  // extern "C"
