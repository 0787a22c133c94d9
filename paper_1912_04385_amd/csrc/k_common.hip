// Shared device utilities: prefix scan, fills, pattern checks, conversions.
#include "internal.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

namespace cptr {

// ---------------------------------------------------------------------------
// caching device allocator
// ---------------------------------------------------------------------------
static thread_local hipStream_t t_stream = nullptr;
static std::mutex g_pool_mu;
static std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void *>> *g_pool;

hipStream_t current_stream() { return t_stream; }

StreamScope::StreamScope(hipStream_t s) : prev(t_stream) { t_stream = s; }
StreamScope::~StreamScope() { t_stream = prev; }

static size_t round_cap(size_t bytes) {
    // 256-byte granules, then at most 1/8 slack per power of two
    size_t b = (bytes + 255) & ~(size_t)255;
    if (b <= 4096) return b;
    size_t p2 = 1;
    while (p2 < b) p2 <<= 1;
    size_t step = p2 / 16;
    return ((b + step - 1) / step) * step;
}

void *pool_alloc(size_t bytes, size_t *cap, hipStream_t *owner, int *devp) {
    int dev = 0;
    CPTR_HIP(hipGetDevice(&dev));
    *devp = dev;
    const size_t want = round_cap(bytes);
    const hipStream_t s = t_stream;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (!g_pool) g_pool = new std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void *>>();
        auto &fl = (*g_pool)[{dev, s}];
        auto it = fl.lower_bound(want);
        if (it != fl.end() && it->first <= want + want / 4) {
            void *p = it->second;
            *cap = it->first;
            fl.erase(it);
            *owner = s;
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        // give idle blocks of this stream back and retry once
        (void)hipGetLastError();
        pool_trim(s);
        CPTR_HIP(hipMalloc(&p, want));
    }
    *cap = want;
    *owner = s;
    return p;
}

void pool_free(void *p, size_t cap, hipStream_t owner, int dev) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    if (!g_pool) g_pool = new std::map<std::pair<int, hipStream_t>, std::multimap<size_t, void *>>();
    (*g_pool)[{dev, owner}].insert({cap, p});
}

void pool_trim(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::multimap<size_t, void *> victims;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (!g_pool) return;
        auto it = g_pool->find({dev, s});
        if (it == g_pool->end()) return;
        victims.swap(it->second);
    }
    (void)hipStreamSynchronize(s);
    for (auto &kv : victims) (void)hipFree(kv.second);
}

// 256-thread blocks: they find room on the GPU beside concurrent kernels
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// exclusive scan of one value per thread across a 1024-thread block
__device__ inline int block_scan_excl(int v, int *lds_waves, int *total) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds_waves[wave] = x;
    __syncthreads();
    if (wave == 0) {
        int w = (lane < (int)(blockDim.x >> 6)) ? lds_waves[lane] : 0;
        int s = w;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int y = __shfl_up(s, d, 64);
            if (lane >= d) s += y;
        }
        if (lane < (int)(blockDim.x >> 6)) lds_waves[lane] = s - w;
        if (lane == (int)(blockDim.x >> 6) - 1) lds_waves[32] = s;
    }
    __syncthreads();
    int r = x - v + lds_waves[wave];
    if (total) *total = lds_waves[32];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_blocksum(const int *in, int n, int *bsum) {
    __shared__ int lds[33];
    long base = (long)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) s += in[base + k];
    int tot;
    block_scan_excl(s, lds, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_offsets(int *bsum, int nb, int *out_total, int *out_total2) {
    __shared__ int lds[33];
    int carry = 0;
    for (int base = 0; base < nb; base += SCAN_THREADS) {
        int i = base + threadIdx.x;
        int v = (i < nb) ? bsum[i] : 0;
        int tot;
        int e = block_scan_excl(v, lds, &tot);
        if (i < nb) bsum[i] = e + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *out_total = carry;
        if (out_total2) *out_total2 = carry;
    }
}

// the whole scan in one block, tile after tile (short inputs); wider tiles
// than the multi-block scan's, so that the chain of tiles stays short: each
// thread takes SCAN1_ITEMS consecutive values, their loads issued together
constexpr int SCAN1_ITEMS = 32;
constexpr int SCAN1_TILE = SCAN_THREADS * SCAN1_ITEMS;

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_single(const int *in, int n, int *out, int *out_total,
                                                              int *out_total2) {
    __shared__ int lds[33];
    int carry = 0;
    for (long t0 = 0; t0 < n; t0 += SCAN1_TILE) {
        const long base = t0 + (long)threadIdx.x * SCAN1_ITEMS;
        int v[SCAN1_ITEMS];
#pragma unroll
        for (int k = 0; k < SCAN1_ITEMS; ++k) v[k] = (base + k < n) ? in[base + k] : 0;
        int sum = 0;
#pragma unroll
        for (int k = 0; k < SCAN1_ITEMS; ++k) sum += v[k];
        int tot;
        int e = block_scan_excl(sum, lds, &tot) + carry;
#pragma unroll
        for (int k = 0; k < SCAN1_ITEMS; ++k) {
            if (base + k < n) out[base + k] = e;
            e += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *out_total = carry;
        if (out_total2) *out_total2 = carry;
    }
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_final(const int *in, int n, const int *boff, int *out) {
    __shared__ int lds[33];
    long base = (long)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int e = block_scan_excl(s, lds, nullptr) + boff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = e;
        e += v[k];
    }
}

// the block sums live in a pooled buffer of the calling stream
// up to this many tiles the scan runs as a single block
constexpr int SCAN_SINGLE_TILES = 32;

void scan_exclusive(const int *in, int *out, int n, int *total_dev, hipStream_t s) {
    int nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nb < 1) nb = 1;
    int *tot = total_dev ? total_dev : out + n;
    int *tot2 = (total_dev && total_dev != out + n) ? out + n : nullptr;
    if (nb <= SCAN_SINGLE_TILES) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(SCAN_THREADS), 0, s, in, n, out, tot, tot2);
        CPTR_CHECK_LAUNCH();
        return;
    }
    DBuf<int> scratch;
    scratch.alloc((size_t)nb + 1);
    int *bsum = scratch.p;
    hipLaunchKernelGGL(k_scan_blocksum, dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(SCAN_THREADS), 0, s, bsum, nb, tot, tot2);
    hipLaunchKernelGGL(k_scan_final, dim3(nb), dim3(SCAN_THREADS), 0, s, in, n, bsum, out);
    CPTR_CHECK_LAUNCH();
}

// Small device-to-host reads: one wavefront copies `bytes` into coherent
// pinned host memory, then publishes `seq` beside them with a system-scope
// release store (every lane's bytes are stored and acknowledged before it),
// so the host can poll the sequence word instead of waiting on the stream.
__global__ void __launch_bounds__(64) k_post_host(const unsigned char *d, int bytes, unsigned char *hdata,
                                                  unsigned long long *hseq, unsigned long long seq) {
    for (int k = threadIdx.x; k < bytes; k += 64) hdata[k] = d[k];
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(hseq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void post_to_host(const void *d, int bytes, void *hdata_dev, unsigned long long *hseq_dev, unsigned long long seq,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_post_host, dim3(1), dim3(64), 0, s, (const unsigned char *)d, bytes,
                       (unsigned char *)hdata_dev, hseq_dev, seq);
    CPTR_CHECK_LAUNCH();
}

// up to four device ints side by side, for one host read
__global__ void k_gather_ints(const int *a, const int *b, const int *c, const int *d, int *out) {
    if (threadIdx.x == 0) {
        out[0] = a ? *a : 0;
        out[1] = b ? *b : 0;
        out[2] = c ? *c : 0;
        out[3] = d ? *d : 0;
    }
}

void gather_ints(const int *a, const int *b, const int *c, int *out, hipStream_t s, const int *d) {
    hipLaunchKernelGGL(k_gather_ints, dim3(1), dim3(64), 0, s, a, b, c, d, out);
    CPTR_CHECK_LAUNCH();
}

template <class T>
__global__ void k_fill(T *p, T v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

static int grid_for(size_t n, int threads, int cap = 65536) {
    size_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > (size_t)cap) g = cap;
    return (int)g;
}

void fill_int(int *p, int v, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<int>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    CPTR_CHECK_LAUNCH();
}

void fill_double(double *p, double v, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
    CPTR_CHECK_LAUNCH();
}

// flag bits: 1 column out of range, 2 columns not ascending, 4 diagonal missing
__global__ void k_check_pattern(int n, const int *rp, const int *ci, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int f = 0, diag = 0, prev = -1;
    int a = rp[i], b = rp[i + 1];
    if (b < a) f |= 2;
    for (int e = a; e < b; ++e) {
        int j = ci[e];
        if (j < 0 || j >= n) f |= 1;
        if (j <= prev) f |= 2;
        if (j == i) diag = 1;
        prev = j;
    }
    if (!diag) f |= 4;
    if (f) atomicOr(flag, f);
}

void check_pattern(int n, const int *rp, const int *ci, int *flag_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_check_pattern, dim3((n + 255) / 256), dim3(256), 0, s, n, rp, ci, flag_dev);
    CPTR_CHECK_LAUNCH();
}

__global__ void k_check_grid5(int n, int nx, const int *rp, const int *ci, int *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int d = ci[e] - i;
        if (d != -nx && d != -1 && d != 0 && d != 1 && d != nx) { atomicOr(flag, 512); return; }
    }
}

void check_grid5(int n, int nx, const int *rp, const int *ci, int *flag_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_check_grid5, dim3((n + 255) / 256), dim3(256), 0, s, n, nx, rp, ci, flag_dev);
    CPTR_CHECK_LAUNCH();
}

// tpos[e] = position of entry (j, i) for e = (i, j); flag bit 8 when missing
__global__ void k_transpose_index(int n, const int *rp, const int *ci, int *tpos, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int j = ci[e];
        int lo = rp[j], hi = rp[j + 1] - 1, pos = -1;
        while (lo <= hi) {
            int mid = (lo + hi) >> 1;
            int c = ci[mid];
            if (c == i) { pos = mid; break; }
            if (c < i) lo = mid + 1; else hi = mid - 1;
        }
        tpos[e] = pos;
        if (pos < 0) atomicOr(flag, 8);
    }
}

void transpose_index(int n, const int *rp, const int *ci, int *tpos, int *flag_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_index, dim3((n + 255) / 256), dim3(256), 0, s, n, rp, ci, tpos, flag_dev);
    CPTR_CHECK_LAUNCH();
}

__global__ void k_nonfinite(const double *x, size_t n, int *flag) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    int bad = 0;
    for (; i < n; i += st)
        if (!isfinite(x[i])) bad = 1;
    if (bad) atomicOr(flag, 16);
}

void count_nonfinite(const double *x, size_t n, int *flag_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, x, n, flag_dev);
    CPTR_CHECK_LAUNCH();
}

__global__ void k_to_float(const double *x, float *y, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) y[i] = (float)x[i];
}

void to_float(const double *x, float *y, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_float, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
    CPTR_CHECK_LAUNCH();
}

// several conversions in one launch: blockIdx.y selects the job (the jobs
// travel in the kernel arguments)
struct ToFloatBatch {
    ToFloatJob j[TF_MAX_JOBS];
};

__global__ void k_to_float_multi(ToFloatBatch b) {
    const ToFloatJob jb = b.j[blockIdx.y];
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t st = (size_t)gridDim.x * blockDim.x;
    for (; i < jb.n; i += st) jb.dst[i] = (float)jb.src[i];
}

void to_float_multi(const ToFloatJob *jobs, int count, hipStream_t s) {
    for (int base = 0; base < count; base += TF_MAX_JOBS) {
        const int k = std::min(TF_MAX_JOBS, count - base);
        ToFloatBatch b{};
        size_t longest = 1;
        for (int q = 0; q < k; ++q) {
            b.j[q] = jobs[base + q];
            longest = std::max(longest, b.j[q].n);
        }
        hipLaunchKernelGGL(k_to_float_multi, dim3(grid_for(longest, 256, 4096), k), dim3(256), 0, s, b);
        CPTR_CHECK_LAUNCH();
    }
}

}  // namespace cptr
