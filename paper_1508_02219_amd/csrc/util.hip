// Device memory cache, prefix sums, fills and small reductions used by every stage.
#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>

#include "common.h"

namespace vb {

// ---------------------------------------------------------------------------------
// Caching allocator.  Sizes are rounded (256 B below 1 MiB, 2 MiB above) and a free block
// is reused for a request on the same stream when it is at most a quarter (or 2 MiB)
// larger, smallest fit first.  When a request misses the cache and would take the memory
// held (in use + cached) above three quarters of the device, or when hipMalloc fails, the
// device is synchronized and every cached block goes back to the runtime first.
// ---------------------------------------------------------------------------------
namespace {
struct DevCache {
    std::mutex mu;
    std::unordered_map<hipStream_t, std::multimap<size_t, void *>> free_by_stream;
    std::unordered_map<void *, size_t> live;
    size_t live_bytes = 0, cached_bytes = 0, peak_bytes = 0;
    size_t budget = 0;  // three quarters of the device memory, read at the first miss
    int64_t runtime_allocs = 0;

    static size_t round_size(size_t b) {
        const size_t small = 256, big = (size_t)2 << 20;
        return b < ((size_t)1 << 20) ? (b + small - 1) / small * small : (b + big - 1) / big * big;
    }
    void release_cached_locked() {
        (void)hipDeviceSynchronize();
        for (auto &kv : free_by_stream)
            for (auto &blk : kv.second) (void)hipFree(blk.second);
        free_by_stream.clear();
        cached_bytes = 0;
    }
};
DevCache &dev_cache() {
    // never destroyed: freeing device memory after the runtime has shut down is unsafe,
    // and the process exit returns everything anyway
    static DevCache *c = new DevCache();
    return *c;
}
}  // namespace

void *dev_alloc(size_t bytes, hipStream_t s) {
    DevCache &c = dev_cache();
    const size_t want = DevCache::round_size(bytes);
    std::lock_guard<std::mutex> lk(c.mu);
    auto fl = c.free_by_stream.find(s);
    if (fl != c.free_by_stream.end()) {
        auto it = fl->second.lower_bound(want);
        const size_t slack = std::max(want / 4, (size_t)2 << 20);
        if (it != fl->second.end() && it->first <= want + slack) {
            void *p = it->second;
            const size_t got = it->first;
            fl->second.erase(it);
            c.cached_bytes -= got;
            c.live[p] = got;
            c.live_bytes += got;
            c.peak_bytes = std::max(c.peak_bytes, c.live_bytes);
            return p;
        }
    }
    if (c.budget == 0) {
        size_t fr = 0, tot = 0;
        c.budget = hipMemGetInfo(&fr, &tot) == hipSuccess && tot > 0 ? tot / 4 * 3 : (size_t)-1;
    }
    if (c.cached_bytes > 0 && c.live_bytes + c.cached_bytes + want > c.budget) c.release_cached_locked();
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        c.release_cached_locked();
        e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(VBARMS_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
    }
    ++c.runtime_allocs;
    c.live[p] = want;
    c.live_bytes += want;
    c.peak_bytes = std::max(c.peak_bytes, c.live_bytes);
    return p;
}

void dev_free(void *p, hipStream_t s) {
    if (!p) return;
    DevCache &c = dev_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.live.find(p);
    if (it == c.live.end()) return;  // not ours: never happens for DBuf
    const size_t b = it->second;
    c.live.erase(it);
    c.live_bytes -= b;
    c.free_by_stream[s].emplace(b, p);
    c.cached_bytes += b;
}

void *pinned_staging(size_t bytes) {
    struct Staging {
        void *p = nullptr;
        size_t n = 0;
    };
    // one buffer per host thread; it is not freed at thread exit, since the runtime may be
    // torn down before thread-local destructors run
    static thread_local Staging st;
    if (bytes > st.n) {
        if (st.p) (void)hipHostFree(st.p);
        st.p = nullptr;
        st.n = 0;
        const size_t want = std::max(bytes + bytes / 2, (size_t)1 << 20);
        if (hipHostMalloc(&st.p, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            st.p = nullptr;
            fail(VBARMS_ERR_OOM, "pinned host allocation of " + std::to_string(want) + " bytes failed");
        }
        st.n = want;
    }
    return st.p;
}

DevCacheStats dev_cache_stats() {
    DevCache &c = dev_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    return DevCacheStats{c.live_bytes, c.cached_bytes, c.peak_bytes, c.runtime_allocs};
}

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
    DBuf<int64_t> tbuf(2 * ntiles + 2);
    int64_t *tsum = tbuf.p;
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
    DBuf<int> d(1);
    fill_i32(d.p, 0, 1, s);
    k_max_block<<<grid_for(p, 256), 256, 0, s>>>(rb, p, d.p);
    VB_LAUNCH_CHECK();
    return read_one(d.p, s);
}

}  // namespace vb
