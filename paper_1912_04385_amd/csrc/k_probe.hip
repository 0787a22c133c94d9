// The streaming-read rate of the GPU's HBM, the practical ceiling of the
// solver's bandwidth-bound kernels: a hand-written kernel that reads a
// buffer once with the access pattern of the outer SpMV's value stream
// (non-temporal 8-byte loads, each wavefront covering 512 contiguous bytes
// per load, several loads in flight per lane) and writes one partial sum per
// workgroup.
#include "internal.h"

namespace cptr {

constexpr int SR_THREADS = 256;
constexpr int SR_UNROLL = 8;
constexpr int SR_MAX_BLOCKS = 4096;

__global__ void __launch_bounds__(SR_THREADS) k_stream_read(size_t n, const double *__restrict__ x,
                                                            double *__restrict__ part) {
    __shared__ double red[SR_THREADS / 64];
    const size_t stride = (size_t)gridDim.x * SR_THREADS;
    const size_t tid = (size_t)blockIdx.x * SR_THREADS + threadIdx.x;
    double acc = 0.0;
    size_t i = tid;
    for (; i + (SR_UNROLL - 1) * stride < n; i += SR_UNROLL * stride) {
        double v[SR_UNROLL];
#pragma unroll
        for (int u = 0; u < SR_UNROLL; ++u) v[u] = __builtin_nontemporal_load(x + i + u * stride);
#pragma unroll
        for (int u = 0; u < SR_UNROLL; ++u) acc += v[u];
    }
    for (; i < n; i += stride) acc += __builtin_nontemporal_load(x + i);
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
    const size_t per = (size_t)SR_THREADS * SR_UNROLL;
    size_t g = (n + per - 1) / per;
    return (int)std::max<size_t>(1, std::min<size_t>(g, SR_MAX_BLOCKS));
}

void launch_stream_read(size_t n, const double *x, double *part, hipStream_t s) {
    hipLaunchKernelGGL(k_stream_read, dim3(stream_read_blocks(n)), dim3(SR_THREADS), 0, s, n, x, part);
    CPTR_CHECK_LAUNCH();
}

}  // namespace cptr
