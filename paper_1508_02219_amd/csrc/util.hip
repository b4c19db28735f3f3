// Prefix sums, fills and small reductions used by every stage.
#include "common.h"

namespace vb {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

template <class Tin, class Tout>
__global__ void __launch_bounds__(kScanThreads) k_scan_tile(const Tin *in, Tout *out, int64_t *tile_sum, int64_t n) {
    __shared__ int64_t sh[kScanThreads];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanItems;
    int64_t v[kScanItems];
    int64_t loc = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = (base + j < n) ? (int64_t)in[base + j] : 0;
        loc += v[j];
    }
    sh[t] = loc;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int64_t x = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    int64_t run = sh[t] - loc;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = (Tout)run;
        run += v[j];
    }
    if (t == kScanThreads - 1) tile_sum[blockIdx.x] = sh[t];
}

template <class Tout>
__global__ void k_scan_add(Tout *out, const int64_t *tile_off, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (Tout)((int64_t)out[i] + tile_off[i / kScanTile]);
}

template <class Tout>
__global__ void k_scan_total(Tout *out, const int64_t *tile_off, int64_t n, int64_t ntiles) {
    out[n] = (Tout)tile_off[ntiles];
}

// exclusive scan of in[0..n) into out[0..n], out[n] = total
template <class Tin, class Tout>
void scan_impl(const Tin *in, Tout *out, int64_t n, hipStream_t s) {
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles == 0) ntiles = 1;
    int64_t *tsum = nullptr;
    VB_HIP(hipMallocAsync((void **)&tsum, sizeof(int64_t) * (2 * ntiles + 2), s));
    int64_t *toff = tsum + ntiles + 1;
    k_scan_tile<Tin, Tout><<<(unsigned)ntiles, kScanThreads, 0, s>>>(in, out, tsum, n);
    VB_LAUNCH_CHECK();
    if (ntiles > 1) {
        scan_impl<int64_t, int64_t>(tsum, toff, ntiles, s);
        k_scan_add<Tout><<<grid_for(n, 256), 256, 0, s>>>(out, toff, n);
        VB_LAUNCH_CHECK();
    } else {
        // toff = {0, tsum[0]}
        VB_HIP(hipMemsetAsync(toff, 0, sizeof(int64_t), s));
        VB_HIP(hipMemcpyAsync(toff + 1, tsum, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    }
    k_scan_total<Tout><<<1, 1, 0, s>>>(out, toff, n, ntiles);
    VB_LAUNCH_CHECK();
    VB_HIP(hipFreeAsync(tsum, s));
}

template <class T>
__global__ void k_fill(T *p, T v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_iota(int *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int)i;
}
__global__ void k_rowblk(const int *rb, int p, int *rowblk) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    for (int r = rb[I]; r < rb[I + 1]; ++r) rowblk[r] = I;
}
__global__ void k_max_block(const int *rb, int p, int *out) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= p) return;
    atomicMax(out, rb[I + 1] - rb[I]);
}

}  // namespace

int64_t scan_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t s, bool want_total) {
    scan_impl<int64_t, int64_t>(in, out, n, s);
    return want_total ? read_one(out + n, s) : 0;
}
int64_t scan_i32_to_i64(const int *in, int64_t *out, int64_t n, hipStream_t s, bool want_total) {
    scan_impl<int, int64_t>(in, out, n, s);
    return want_total ? read_one(out + n, s) : 0;
}
int scan_i32(const int *in, int *out, int64_t n, hipStream_t s, bool want_total) {
    scan_impl<int, int>(in, out, n, s);
    return want_total ? read_one(out + n, s) : 0;
}
void fill_i32(int *p, int v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<int><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    VB_LAUNCH_CHECK();
}
void fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<int64_t><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    VB_LAUNCH_CHECK();
}
template <class T>
void fill_val(T *p, T v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<T><<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    VB_LAUNCH_CHECK();
}
template void fill_val<double>(double *, double, int64_t, hipStream_t);
template void fill_val<float>(float *, float, int64_t, hipStream_t);
template void fill_val<unsigned long long>(unsigned long long *, unsigned long long, int64_t, hipStream_t);

void iota_i32(int *p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_iota<<<grid_for(n, 256), 256, 0, s>>>(p, n);
    VB_LAUNCH_CHECK();
}
void fill_rowblk(const int *rb, int p, int *rowblk, hipStream_t s) {
    if (p <= 0) return;
    k_rowblk<<<grid_for(p, 256), 256, 0, s>>>(rb, p, rowblk);
    VB_LAUNCH_CHECK();
}
int max_block_size(const int *rb, int p, hipStream_t s) {
    if (p <= 0) return 0;
    int *d = nullptr;
    VB_HIP(hipMallocAsync((void **)&d, sizeof(int), s));
    VB_HIP(hipMemsetAsync(d, 0, sizeof(int), s));
    k_max_block<<<grid_for(p, 256), 256, 0, s>>>(rb, p, d);
    VB_LAUNCH_CHECK();
    int m = read_one(d, s);
    VB_HIP(hipFreeAsync(d, s));
    return m;
}

}  // namespace vb
