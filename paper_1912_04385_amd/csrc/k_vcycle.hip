// AMG V-cycle pieces for the scalar stages (M_TT^{-1} = amg(C_TT),
// M_PP^{-1} = amg(B_PP)) and the scalar glue of Algorithm 2.  Templated on the
// working precision (double, or float for the precision-split preconditioner).
// Scalar CSR rows are short (5 on the fine level); these kernels use one
// thread per row and are bound by HBM traffic of the CSR arrays and vectors.
#include "internal.h"

namespace cptr {

static inline int nblocks(long n, int t) { long b = (n + t - 1) / t; return (int)(b < 1 ? 1 : b); }

// first Jacobi sweep from a zero guess fused with the residual:
//   x_i = omega dinv_i b_i,   r_i = b_i - sum_j a_ij (omega dinv_j b_j)
template <class T>
__global__ void k_presmooth_residual(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                     const T *__restrict__ v, const T *__restrict__ dinv, T omega,
                                     const T *__restrict__ b, T *__restrict__ x, T *__restrict__ r) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int j = ci[e];
        acc += v[e] * (omega * dinv[j] * b[j]);
    }
    const T bi = b[i];
    x[i] = omega * dinv[i] * bi;
    r[i] = bi - acc;
}

template <class T>
void vc_presmooth_residual(int n, const int *rp, const int *ci, const T *v, const T *dinv, T omega, const T *b,
                           int bstride, int boff, T *x, T *r, hipStream_t st) {
    (void)bstride; (void)boff;
    if (n == 0) return;
    hipLaunchKernelGGL(k_presmooth_residual<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, rp, ci, v, dinv, omega,
                       b, x, r);
    CPTR_CHECK_LAUNCH();
}

// y = A x
template <class T>
__global__ void k_spmv(int n, const int *__restrict__ rp, const int *__restrict__ ci, const T *__restrict__ v,
                       const T *__restrict__ x, T *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) acc += v[e] * x[ci[e]];
    y[i] = acc;
}

template <class T>
void vc_spmv(int n, const int *rp, const int *ci, const T *v, const T *x, T *y, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_spmv<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, rp, ci, v, x, y);
    CPTR_CHECK_LAUNCH();
}

// xout = xin + P xc (xout may alias xin)
template <class T>
__global__ void k_prolong_add(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                              const T *__restrict__ v, const T *__restrict__ xc, const T *xin, T *xout) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = xin[i];
    for (int e = rp[i]; e < rp[i + 1]; ++e) acc += v[e] * xc[ci[e]];
    xout[i] = acc;
}

template <class T>
void vc_prolong_add(int n, const int *rp, const int *ci, const T *v, const T *xc, T *x, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_prolong_add<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, rp, ci, v, xc, x, x);
    CPTR_CHECK_LAUNCH();
}

template <class T>
void vc_prolong_to(int n, const int *rp, const int *ci, const T *v, const T *xc, const T *xin, T *xout,
                   hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_prolong_add<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, rp, ci, v, xc, xin, xout);
    CPTR_CHECK_LAUNCH();
}

// one damped Jacobi sweep: xout = xin + omega dinv (b - A xin)
template <class T>
__global__ void k_smooth(int n, const int *__restrict__ rp, const int *__restrict__ ci, const T *__restrict__ v,
                         const T *__restrict__ dinv, T omega, const T *__restrict__ b, const T *__restrict__ xin,
                         T *__restrict__ xout) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) acc += v[e] * xin[ci[e]];
    xout[i] = xin[i] + omega * dinv[i] * (b[i] - acc);
}

template <class T>
void vc_smooth(int n, const int *rp, const int *ci, const T *v, const T *dinv, T omega, const T *b, int bstride,
               int boff, const T *xin, T *xout, hipStream_t st) {
    (void)bstride; (void)boff;
    if (n == 0) return;
    hipLaunchKernelGGL(k_smooth<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, rp, ci, v, dinv, omega, b, xin,
                       xout);
    CPTR_CHECK_LAUNCH();
}

// r = b - A x
template <class T>
__global__ void k_residual(int n, const int *__restrict__ rp, const int *__restrict__ ci, const T *__restrict__ v,
                           const T *__restrict__ b, const T *__restrict__ x, T *__restrict__ r) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) acc += v[e] * x[ci[e]];
    r[i] = b[i] - acc;
}

template <class T>
void vc_residual(int n, const int *rp, const int *ci, const T *v, const T *b, const T *x, T *r, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_residual<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, rp, ci, v, b, x, r);
    CPTR_CHECK_LAUNCH();
}

// coarsest level: x = Ainv b (dense, one wavefront per row); accumulation in
// double in both precisions (the coarse solve stays FP64)
template <class T>
__global__ void __launch_bounds__(256) k_dense_apply(int n, const T *__restrict__ M, const T *__restrict__ b,
                                                     T *__restrict__ x) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double acc = 0.0;
    for (int c = lane; c < n; c += 64) acc += (double)M[(size_t)row * n + c] * (double)b[c];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) x[row] = (T)acc;
}

template <class T>
void vc_dense_apply(int n, const T *Minv, const T *b, T *x, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_dense_apply<T>, dim3((n + 3) / 4), dim3(256), 0, st, n, Minv, b, x);
    CPTR_CHECK_LAUNCH();
}

// the coarsest solve of the FP32 preconditioner stays FP64: cast in, apply, cast out
__global__ void __launch_bounds__(256) k_dense_apply_mixed(int n, const double *__restrict__ M,
                                                           const float *__restrict__ b, float *__restrict__ x) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double acc = 0.0;
    for (int c = lane; c < n; c += 64) acc += M[(size_t)row * n + c] * (double)b[c];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) x[row] = (float)acc;
}

void vc_dense_apply_mixed(int n, const double *Minv, const float *b, float *x, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_dense_apply_mixed, dim3((n + 3) / 4), dim3(256), 0, st, n, Minv, b, x);
    CPTR_CHECK_LAUNCH();
}

// Algorithm 2 glue: out_i = r[i*b + comp] - sum_e slab[e*b + comp] * xs[ci[e]]
// (z_P = r_P - Abar[P,T] x_T when the T stage runs first)
template <class T>
__global__ void k_stage_input(int n, int b, const int *__restrict__ rp, const int *__restrict__ ci,
                              const T *__restrict__ slab, int comp, const double *__restrict__ r,
                              const T *__restrict__ xs, T *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = (T)r[(size_t)i * b + comp];
    if (xs)
        for (int e = rp[i]; e < rp[i + 1]; ++e) acc -= slab[(size_t)e * b + comp] * xs[ci[e]];
    out[i] = acc;
}

template <class T>
void ms_stage_input(int n, int b, const int *rp, const int *ci, const T *slab, int comp, const double *r,
                    const T *xs, T *out, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_stage_input<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, b, rp, ci, slab, comp, r, xs,
                       out);
    CPTR_CHECK_LAUNCH();
}

// start vector of the convergence-factor measurement: SplitMix64 of
// (seed, i) mapped to a uniform double in [-1, 1) (53 random bits, exact)
__device__ inline uint64_t vc_splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void k_hash_uniform(int n, uint64_t seed, double *__restrict__ e) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t u = vc_splitmix64(seed, (uint64_t)i);
    e[i] = (double)(u >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

void vc_hash_uniform(int n, uint64_t seed, double *e, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_hash_uniform, dim3(nblocks(n, 256)), dim3(256), 0, st, n, seed, e);
    CPTR_CHECK_LAUNCH();
}

// e -= x
__global__ void k_sub(int n, const double *__restrict__ x, double *__restrict__ e) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) e[i] -= x[i];
}

void vc_sub(int n, const double *x, double *e, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_sub, dim3(nblocks(n, 256)), dim3(256), 0, st, n, x, e);
    CPTR_CHECK_LAUNCH();
}

#define INST(T)                                                                                                   \
    template void vc_presmooth_residual<T>(int, const int *, const int *, const T *, const T *, T, const T *, int, \
                                           int, T *, T *, hipStream_t);                                          \
    template void vc_spmv<T>(int, const int *, const int *, const T *, const T *, T *, hipStream_t);             \
    template void vc_prolong_add<T>(int, const int *, const int *, const T *, const T *, T *, hipStream_t);      \
    template void vc_prolong_to<T>(int, const int *, const int *, const T *, const T *, const T *, T *,          \
                                   hipStream_t);                                                                 \
    template void vc_smooth<T>(int, const int *, const int *, const T *, const T *, T, const T *, int, int,        \
                               const T *, T *, hipStream_t);                                                     \
    template void vc_residual<T>(int, const int *, const int *, const T *, const T *, const T *, T *,            \
                                 hipStream_t);                                                                   \
    template void vc_dense_apply<T>(int, const T *, const T *, T *, hipStream_t);                                \
    template void ms_stage_input<T>(int, int, const int *, const int *, const T *, int, const double *,          \
                                    const T *, T *, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace cptr
