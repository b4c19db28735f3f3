// Parameter prediction: matrix features and a small FP32 multilayer perceptron.
//
// The network maps a feature vector of the matrix to the compression threshold tau and
// the per-level drop tolerances.  It is trained on sweeps the method itself runs, so the
// forward pass, backpropagation and the Adam update are kernels here.  Layers are
// 128 wide and batches small, so every dense layer is a plain FP32 kernel (one thread
// per output element, fixed summation order, deterministic); matrix cores would sit
// mostly idle at these shapes.
//
// Parameters are packed layer by layer: W_l (n_out x n_in, row-major), then b_l (n_out).
// Loss: sum over batch and outputs of (y - t)^2 / (B * n_out).
#include <cmath>

#include "factor.h"

struct vbarms_mlp_ctx {
    int in_dim = 0, hidden = 0, depth = 0, out_dim = 0;
    int nlayers = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    std::string last_error;
    std::vector<int> nin, nout;         // per layer
    std::vector<int64_t> woff, boff;    // parameter offsets per layer
    int64_t nparams = 0;
    vb::DBuf<float> params, grads, m1, m2;
    vb::DBuf<float> xs;                 // inputs of layers 1.., B x sum(n_in) (layer 0 reads x)
    vb::DBuf<float> zs;                 // pre-activations, B x sum(n_out)
    vb::DBuf<float> dz0, dz1;           // back-propagated gradients, B x max width
    vb::DBuf<float> loss;               // [1]
    std::vector<int64_t> xoff, zoff;    // per-layer offsets (in elements per sample)
    int64_t xw = 0, zw = 0;             // widths of xs and zs per sample
    int maxw = 0;
    int cap = 0;                        // batch capacity of the workspaces
    int64_t steps = 0;                  // Adam steps taken
    bool have_grad = false;
};

namespace vb {
namespace {

constexpr int kMlpThreads = 128;

// Z[b, o] = b_o + sum_i W[o, i] X[b, i]; A[b, o] = ReLU(Z) or Z.  One block per sample.
__global__ void __launch_bounds__(kMlpThreads) k_dense_fwd(int nin, int nout, const float *W, const float *bias,
                                                           const float *X, int64_t ldx, float *Z, int64_t ldz,
                                                           float *A, int64_t lda, int relu) {
    extern __shared__ float xrow[];
    const int b = blockIdx.x;
    for (int i = threadIdx.x; i < nin; i += kMlpThreads) xrow[i] = X[(int64_t)b * ldx + i];
    __syncthreads();
    for (int o = threadIdx.x; o < nout; o += kMlpThreads) {
        const float *w = W + (int64_t)o * nin;
        float z = bias[o];
        for (int i = 0; i < nin; ++i) z = z + w[i] * xrow[i];
        if (Z) Z[(int64_t)b * ldz + o] = z;
        A[(int64_t)b * lda + o] = relu ? fmaxf(z, 0.0f) : z;
    }
}

// dY = 2 (Y - T) / (B n); loss = sum (Y - T)^2 / (B n), reduced in a fixed order by one block.
__global__ void __launch_bounds__(256) k_mse(int B, int n, const float *Y, int64_t ldy, const float *T, float *dY,
                                             int64_t lddy, float *loss) {
    __shared__ float part[256];
    const float scale = 1.0f / ((float)B * (float)n);
    float s = 0.0f;
    for (int e = threadIdx.x; e < B * n; e += 256) {
        int b = e / n, o = e % n;
        float d = Y[(int64_t)b * ldy + o] - T[e];
        dY[(int64_t)b * lddy + o] = 2.0f * d * scale;
        s = s + d * d;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float tot = 0.0f;
        for (int k = 0; k < 256; ++k) tot = tot + part[k];
        *loss = tot * scale;
    }
}

// dX[b, i] = sum_o dZ[b, o] W[o, i], times the ReLU derivative of the layer below (Zp > 0).
__global__ void k_dense_bwd_data(int B, int nin, int nout, const float *W, const float *dZ, int64_t lddz,
                                 const float *Zp, int64_t ldzp, float *dX, int64_t lddx) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * nin) return;
    int b = (int)(e / nin), i = (int)(e % nin);
    float s = 0.0f;
    for (int o = 0; o < nout; ++o) s = s + dZ[(int64_t)b * lddz + o] * W[(int64_t)o * nin + i];
    dX[(int64_t)b * lddx + i] = Zp[(int64_t)b * ldzp + i] > 0.0f ? s : 0.0f;
}

// dW[o, i] = sum_b dZ[b, o] X[b, i]; db[o] = sum_b dZ[b, o] (thread i == nin).
__global__ void k_dense_bwd_weights(int B, int nin, int nout, const float *dZ, int64_t lddz, const float *X,
                                    int64_t ldx, float *dW, float *db) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nout * (nin + 1)) return;
    int o = (int)(e / (nin + 1)), i = (int)(e % (nin + 1));
    float s = 0.0f;
    if (i < nin) {
        for (int b = 0; b < B; ++b) s = s + dZ[(int64_t)b * lddz + o] * X[(int64_t)b * ldx + i];
        dW[(int64_t)o * nin + i] = s;
    } else {
        for (int b = 0; b < B; ++b) s = s + dZ[(int64_t)b * lddz + o];
        db[o] = s;
    }
}

// Adam with bias correction: bc1 = 1 - beta1^t, bc2 = 1 - beta2^t.
__global__ void k_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float gi = g[e];
    float mi = b1 * m[e] + (1.0f - b1) * gi;
    float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    float mh = mi / bc1, vh = vi / bc2;
    p[e] = p[e] - lr * mh / (sqrtf(vh) + eps);
}

// ---- matrix features ------------------------------------------------------------------
// Per row: length, |a_ii| / sum_j |a_ij|, count of entries below 1e-3 max_j |a_ij|, the
// mean off-diagonal magnitude over |a_ii|.
__global__ void k_row_features(int n, const int64_t *rowptr, const int *col, const double *val, double *rl,
                               double *dom, double *tiny, double *coup) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int64_t b = rowptr[r], e = rowptr[r + 1];
    double sum = 0.0, mx = 0.0, diag = 0.0, off = 0.0;
    for (int64_t k = b; k < e; ++k) {
        double a = fabs(val[k]);
        sum += a;
        mx = fmax(mx, a);
        if (col[k] == r) diag = a;
        else off += a;
    }
    int64_t cnt = e - b, small = 0;
    for (int64_t k = b; k < e; ++k)
        if (fabs(val[k]) < 1e-3 * mx) ++small;
    rl[r] = (double)cnt;
    dom[r] = sum > 0.0 ? diag / sum : 0.0;
    tiny[r] = (double)small;
    coup[r] = (diag > 0.0 && cnt > 1) ? off / ((double)(cnt - 1) * diag) : 0.0;
}

// column-wise sums / sums of squares / minimum of k double arrays of length n (one block each)
__global__ void __launch_bounds__(256) k_feature_reduce(int n, const double *a, double *out) {
    __shared__ double s1[256], s2[256], s3[256];
    const double *x = a + (int64_t)blockIdx.x * n;
    double sum = 0.0, sq = 0.0, mn = 1e300;
    for (int i = threadIdx.x; i < n; i += 256) {
        double v = x[i];
        sum += v;
        sq += v * v;
        mn = fmin(mn, v);
    }
    s1[threadIdx.x] = sum;
    s2[threadIdx.x] = sq;
    s3[threadIdx.x] = mn;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a1 = 0.0, a2 = 0.0, a3 = 1e300;
        for (int k = 0; k < 256; ++k) {
            a1 += s1[k];
            a2 += s2[k];
            a3 = fmin(a3, s3[k]);
        }
        out[3 * blockIdx.x + 0] = a1;
        out[3 * blockIdx.x + 1] = a2;
        out[3 * blockIdx.x + 2] = a3;
    }
}

}  // namespace

// Features of the matrix (VBARMS_NFEAT values): see vbarms.h.
void matrix_features(int n, int64_t nnz, const int64_t *rowptr, const int *col, const double *val, float *f,
                     hipStream_t s) {
    if (n <= 0) fail(VBARMS_ERR_ARG, "empty matrix");
    DBuf<double> rows(4 * (size_t)n), red(12);
    k_row_features<<<grid_for(n, 256), 256, 0, s>>>(n, rowptr, col, val, rows.p, rows.p + n, rows.p + 2 * (size_t)n,
                                                     rows.p + 3 * (size_t)n);
    VB_LAUNCH_CHECK();
    k_feature_reduce<<<4, 256, 0, s>>>(n, rows.p, red.p);
    VB_LAUNCH_CHECK();
    std::vector<double> r;
    to_host(r, red.p, 12, s);
    // identical-pattern classes (the tau = 1 partition)
    DBuf<int> perm(n);
    std::vector<int> bptr = compress_gpu(n, rowptr, col, 1.0, perm.p, s);
    const double dn = (double)n;
    const double mean_len = r[0] / dn;
    const double var_len = std::max(0.0, r[1] / dn - mean_len * mean_len);
    f[0] = (float)std::log10(dn);
    f[1] = (float)(mean_len / 100.0);
    f[2] = (float)(mean_len > 0.0 ? std::sqrt(var_len) / mean_len : 0.0);
    f[3] = (float)(r[3] / dn);                        // mean diagonal share
    f[4] = (float)r[5];                               // smallest diagonal share
    f[5] = (float)(r[6] / std::max<double>(1.0, (double)nnz));  // share of tiny entries
    f[6] = (float)((double)(bptr.size() - 1) / dn);   // classes per row (1 / block size at tau = 1)
    f[7] = (float)(r[9] / dn);                        // mean coupling over the diagonal
}

}  // namespace vb

using namespace vb;

namespace {

template <class F>
int mlp_guarded(vbarms_mlp_t m, F &&body) {
    if (!m) return VBARMS_ERR_ARG;
    StreamScope scope(m->stream);
    try {
        m->last_error.clear();
        VB_HIP(hipSetDevice(m->device));
        return body();
    } catch (const VbError &e) {
        m->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        m->last_error = "host allocation failed";
        return VBARMS_ERR_OOM;
    } catch (...) {
        m->last_error = "unexpected internal error";
        return VBARMS_ERR_HIP;
    }
}

void ensure_batch(vbarms_mlp_t m, int B) {
    if (B <= m->cap) return;
    m->xs.alloc((size_t)B * m->xw);
    m->zs.alloc((size_t)B * m->zw);
    m->dz0.alloc((size_t)B * m->maxw);
    m->dz1.alloc((size_t)B * m->maxw);
    m->cap = B;
}

// input of layer l: the caller's x for the first layer, else the workspace
const float *layer_in(vbarms_mlp_t m, const float *x, int l, int64_t *ld) {
    if (l == 0) {
        *ld = m->in_dim;
        return x;
    }
    *ld = m->xw;
    return m->xs.p + m->xoff[l];
}

// forward pass; layer inputs and pre-activations stay in the workspaces for the backward pass
void run_forward(vbarms_mlp_t m, const float *x, int B, float *y_out) {
    hipStream_t s = m->stream;
    ensure_batch(m, B);
    for (int l = 0; l < m->nlayers; ++l) {
        const bool last = l == m->nlayers - 1;
        int64_t ldx = 0;
        const float *Xl = layer_in(m, x, l, &ldx);
        float *Zl = m->zs.p + m->zoff[l];
        float *A = last ? y_out : m->xs.p + m->xoff[l + 1];
        int64_t lda = last ? m->out_dim : m->xw;
        k_dense_fwd<<<B, kMlpThreads, sizeof(float) * m->nin[l], s>>>(
            m->nin[l], m->nout[l], m->params.p + m->woff[l], m->params.p + m->boff[l], Xl, ldx, Zl, m->zw, A, lda,
            last ? 0 : 1);
        VB_LAUNCH_CHECK();
    }
}

}  // namespace

extern "C" {

int vbarms_mlp_create(vbarms_mlp_t *out, int32_t in_dim, int32_t hidden, int32_t depth, int32_t out_dim,
                      void *hip_stream) {
    if (!out) return VBARMS_ERR_ARG;
    *out = nullptr;
    if (in_dim < 1 || out_dim < 1 || depth < 0 || depth > 8 || (depth > 0 && hidden < 1) || in_dim > 4096 ||
        hidden > 4096 || out_dim > 4096)
        return VBARMS_ERR_ARG;
    vbarms_mlp_t m = new (std::nothrow) vbarms_mlp_ctx();
    if (!m) return VBARMS_ERR_OOM;
    if (hipGetDevice(&m->device) != hipSuccess) { delete m; return VBARMS_ERR_HIP; }
    m->stream = (hipStream_t)hip_stream;
    m->in_dim = in_dim;
    m->hidden = hidden;
    m->depth = depth;
    m->out_dim = out_dim;
    int rc = mlp_guarded(m, [&] {
        std::vector<int> dims;
        dims.push_back(in_dim);
        for (int d = 0; d < depth; ++d) dims.push_back(hidden);
        dims.push_back(out_dim);
        m->nlayers = (int)dims.size() - 1;
        int64_t off = 0, xo = 0, zo = 0;
        for (int l = 0; l < m->nlayers; ++l) {
            m->nin.push_back(dims[l]);
            m->nout.push_back(dims[l + 1]);
            m->woff.push_back(off);
            off += (int64_t)dims[l + 1] * dims[l];
            m->boff.push_back(off);
            off += dims[l + 1];
            m->xoff.push_back(xo);
            xo += dims[l];
            m->zoff.push_back(zo);
            zo += dims[l + 1];
            m->maxw = std::max(m->maxw, std::max(dims[l], dims[l + 1]));
        }
        m->nparams = off;
        m->xw = xo;
        m->zw = zo;
        m->params.alloc(off);
        m->grads.alloc(off);
        m->m1.alloc(off);
        m->m2.alloc(off);
        m->loss.alloc(1);
        fill_val<float>(m->params.p, 0.0f, off, m->stream);
        fill_val<float>(m->m1.p, 0.0f, off, m->stream);
        fill_val<float>(m->m2.p, 0.0f, off, m->stream);
        VB_HIP(hipStreamSynchronize(m->stream));
        return VBARMS_OK;
    });
    if (rc != VBARMS_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return VBARMS_OK;
}

int vbarms_mlp_destroy(vbarms_mlp_t m) {
    if (!m) return VBARMS_ERR_ARG;
    (void)hipSetDevice(m->device);
    hipStream_t s = m->stream;
    {
        StreamScope scope(s);
        delete m;
    }
    (void)hipStreamSynchronize(s);
    return VBARMS_OK;
}

const char *vbarms_mlp_last_error(vbarms_mlp_t m) { return m ? m->last_error.c_str() : "invalid handle"; }

int vbarms_mlp_num_params(vbarms_mlp_t m, int64_t *n) {
    if (!m || !n) return VBARMS_ERR_ARG;
    *n = m->nparams;
    return VBARMS_OK;
}

int vbarms_mlp_set_params(vbarms_mlp_t m, const float *params) {
    return mlp_guarded(m, [&] {
        if (!params) fail(VBARMS_ERR_ARG, "NULL parameters");
        hipStream_t s = m->stream;
        VB_HIP(hipMemcpyAsync(m->params.p, params, sizeof(float) * m->nparams, hipMemcpyDeviceToDevice, s));
        fill_val<float>(m->m1.p, 0.0f, m->nparams, s);
        fill_val<float>(m->m2.p, 0.0f, m->nparams, s);
        m->steps = 0;
        m->have_grad = false;
        VB_HIP(hipStreamSynchronize(s));
        return VBARMS_OK;
    });
}

int vbarms_mlp_get_params(vbarms_mlp_t m, float *params) {
    return mlp_guarded(m, [&] {
        if (!params) fail(VBARMS_ERR_ARG, "NULL parameters");
        VB_HIP(hipMemcpyAsync(params, m->params.p, sizeof(float) * m->nparams, hipMemcpyDeviceToDevice, m->stream));
        VB_HIP(hipStreamSynchronize(m->stream));
        return VBARMS_OK;
    });
}

int vbarms_mlp_forward(vbarms_mlp_t m, const float *x, int32_t batch, float *y) {
    return mlp_guarded(m, [&] {
        if (batch < 0 || (batch > 0 && (!x || !y))) fail(VBARMS_ERR_ARG, "invalid batch");
        if (batch == 0) return VBARMS_OK;
        run_forward(m, x, batch, y);
        VB_HIP(hipStreamSynchronize(m->stream));
        return VBARMS_OK;
    });
}

int vbarms_mlp_loss_grad(vbarms_mlp_t m, const float *x, const float *t, int32_t batch, float *loss, float *grad) {
    return mlp_guarded(m, [&] {
        if (batch < 1 || !x || !t) fail(VBARMS_ERR_ARG, "invalid batch");
        hipStream_t s = m->stream;
        const int B = batch;
        ensure_batch(m, B);
        DBuf<float> y((size_t)B * m->out_dim);
        run_forward(m, x, B, y.p);
        // output layer gradient, then back through every layer
        float *dz = m->dz0.p, *dzn = m->dz1.p;
        k_mse<<<1, 256, 0, s>>>(B, m->out_dim, y.p, m->out_dim, t, dz, m->maxw, m->loss.p);
        VB_LAUNCH_CHECK();
        for (int l = m->nlayers - 1; l >= 0; --l) {
            const int nin = m->nin[l], nout = m->nout[l];
            int64_t ldx = 0;
            const float *Xl = layer_in(m, x, l, &ldx);
            k_dense_bwd_weights<<<grid_for((int64_t)nout * (nin + 1), 256), 256, 0, s>>>(
                B, nin, nout, dz, m->maxw, Xl, ldx, m->grads.p + m->woff[l], m->grads.p + m->boff[l]);
            VB_LAUNCH_CHECK();
            if (l > 0) {
                const float *Zp = m->zs.p + m->zoff[l - 1];
                k_dense_bwd_data<<<grid_for((int64_t)B * nin, 256), 256, 0, s>>>(B, nin, nout, m->params.p + m->woff[l],
                                                                              dz, m->maxw, Zp, m->zw, dzn, m->maxw);
                VB_LAUNCH_CHECK();
                std::swap(dz, dzn);
            }
        }
        if (grad) VB_HIP(hipMemcpyAsync(grad, m->grads.p, sizeof(float) * m->nparams, hipMemcpyDeviceToDevice, s));
        float h = 0.0f;
        VB_HIP(hipMemcpyAsync(&h, m->loss.p, sizeof(float), hipMemcpyDeviceToHost, s));
        VB_HIP(hipStreamSynchronize(s));
        if (loss) *loss = h;
        m->have_grad = true;
        return VBARMS_OK;
    });
}

int vbarms_mlp_adam_step(vbarms_mlp_t m, float lr) {
    return mlp_guarded(m, [&] {
        if (!m->have_grad) fail(VBARMS_ERR_STATE, "no gradient: call vbarms_mlp_loss_grad first");
        if (!(lr > 0.0f)) fail(VBARMS_ERR_ARG, "learning rate must be positive");
        const double b1 = 0.9, b2 = 0.999;
        m->steps += 1;
        const float bc1 = (float)(1.0 - std::pow(b1, (double)m->steps));
        const float bc2 = (float)(1.0 - std::pow(b2, (double)m->steps));
        k_adam<<<grid_for(m->nparams, 256), 256, 0, m->stream>>>(m->nparams, m->params.p, m->grads.p, m->m1.p, m->m2.p,
                                                                 lr, (float)b1, (float)b2, 1e-8f, bc1, bc2);
        VB_LAUNCH_CHECK();
        VB_HIP(hipStreamSynchronize(m->stream));
        return VBARMS_OK;
    });
}

}  // extern "C"
