// The streaming-read rate of the GPU's HBM, the practical ceiling of the
// solver's bandwidth-bound kernels: a hand-written kernel that reads a
// buffer once with the access pattern of the outer SpMV's value stream
// (non-temporal 16-byte loads, each wavefront covering 1 KB of contiguous
// bytes per load, eight loads in flight per lane, each workgroup streaming
// one contiguous chunk) and writes one partial sum per workgroup.
#include "internal.h"

namespace cptr {

constexpr int SR_THREADS = 256;
constexpr int SR_UNROLL = 8;
constexpr int SR_MAX_BLOCKS = 4096;

typedef double sr_v2d __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(SR_THREADS) k_stream_read(size_t n, const double *__restrict__ x,
                                                            double *__restrict__ part) {
    __shared__ double red[SR_THREADS / 64];
    const sr_v2d *x2 = (const sr_v2d *)x;
    const size_t n2 = n / 2;       // pairs; an odd last element is added by thread 0 of block 0
    // each workgroup reads one contiguous chunk; a pass issues SR_UNROLL
    // loads per lane over SR_UNROLL consecutive 4 KB spans of it
    const size_t chunk = (n2 + gridDim.x - 1) / gridDim.x;
    const size_t c0 = (size_t)blockIdx.x * chunk;
    const size_t c1 = c0 + chunk < n2 ? c0 + chunk : n2;
    double acc = 0.0;
    size_t i = c0 + threadIdx.x;
    for (; i + (SR_UNROLL - 1) * SR_THREADS < c1; i += SR_UNROLL * SR_THREADS) {
        sr_v2d v[SR_UNROLL];
#pragma unroll
        for (int u = 0; u < SR_UNROLL; ++u) v[u] = __builtin_nontemporal_load(x2 + i + u * SR_THREADS);
#pragma unroll
        for (int u = 0; u < SR_UNROLL; ++u) acc += v[u].x + v[u].y;
    }
    for (; i < c1; i += SR_THREADS) {
        const sr_v2d v = __builtin_nontemporal_load(x2 + i);
        acc += v.x + v.y;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) acc += x[n - 1];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < SR_THREADS / 64; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

int stream_read_blocks(size_t n) {
    const size_t per = (size_t)SR_THREADS * SR_UNROLL * 2;
    size_t g = (n + per - 1) / per;
    return (int)std::max<size_t>(1, std::min<size_t>(g, SR_MAX_BLOCKS));
}

void launch_stream_read(size_t n, const double *x, double *part, hipStream_t s) {
    hipLaunchKernelGGL(k_stream_read, dim3(stream_read_blocks(n)), dim3(SR_THREADS), 0, s, n, x, part);
    CPTR_CHECK_LAUNCH();
}

}  // namespace cptr
