// AMG V-cycle pieces for the scalar stages (M_TT^{-1} = amg(C_TT),
// M_PP^{-1} = amg(B_PP)) and the scalar glue of Algorithm 2.  Templated on the
// working precision (double, or float for the precision-split preconditioner).
// Scalar CSR rows are short (5 on the fine level); these kernels use one
// thread per row and are bound by HBM traffic of the CSR arrays and vectors.
#include "internal.h"

namespace cptr {

static inline int nblocks(long n, int t) { long b = (n + t - 1) / t; return (int)(b < 1 ? 1 : b); }

// The level kernels share one row loop: G lanes per row (G = 1 for the short
// rows of the fine level, up to 64 for the long rows of Galerkin coarse
// levels), each lane summing every G-th entry, then an xor-shuffle reduction
// inside the lane group.  OP selects what is done with the row sum
// acc_i = sum_j a_ij x_j:
enum CsrOp {
    OP_SPMV,          // y_i = acc_i                                    (x = xin)
    OP_RESIDUAL,      // r_i = b_i - acc_i                              (x = xin)
    OP_SMOOTH,        // x_i = xin_i + omega dinv_i (b_i - acc_i)       (x = xin)
    OP_PRESMOOTH,     // x_i = omega dinv_i b_i, r_i = b_i - acc_i      (x_j = omega dinv_j b_j)
    OP_PROLONG,       // x_i = xin_i + acc_i                            (x = coarse vector)
    OP_SWEEP_RESID    // x_i = xin_i + omega dinv_i rin_i, r_i = b_i - acc_i
                      //   (x_j = xin_j + omega dinv_j rin_j: the next Jacobi
                      //   sweep from the previous one's residual rin = xs)
};

template <class T, int G, int OP>
__global__ void __launch_bounds__(256) k_csr_op(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                const T *__restrict__ v, const T *__restrict__ xs,
                                                const T *__restrict__ dinv, T omega, const T *__restrict__ b,
                                                const T *xin, T *xout, T *__restrict__ rout) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / G), sub = (int)(t % G);
    const bool act = i < n;
    T acc = 0;
    // single-lane rows of at most ME entries (the fine level): every operand
    // is loaded before the sum, which then runs in row order as below
    constexpr int ME = 8;
    bool done = false;
    if constexpr (G == 1) {
        if (act) {
            const int e0 = rp[i], e1 = rp[i + 1];
            if (e1 - e0 <= ME) {
                int js[ME];
                T vv[ME], o1[ME], o2[ME], o3[ME];
#pragma unroll
                for (int q = 0; q < ME; ++q) js[q] = (e0 + q < e1) ? ci[e0 + q] : 0;
#pragma unroll
                for (int q = 0; q < ME; ++q) {
                    const bool on = e0 + q < e1;
                    const int j = js[q];
                    vv[q] = on ? v[e0 + q] : (T)0;
                    if constexpr (OP == OP_PRESMOOTH) {
                        o1[q] = on ? dinv[j] : (T)0;
                        o2[q] = on ? b[j] : (T)0;
                    } else if constexpr (OP == OP_SWEEP_RESID) {
                        o1[q] = on ? xin[j] : (T)0;
                        o2[q] = on ? dinv[j] : (T)0;
                        o3[q] = on ? xs[j] : (T)0;
                    } else {
                        o1[q] = on ? xs[j] : (T)0;
                    }
                }
#pragma unroll
                for (int q = 0; q < ME; ++q) {
                    if (e0 + q >= e1) break;
                    if constexpr (OP == OP_PRESMOOTH)
                        acc += vv[q] * (omega * o1[q] * o2[q]);
                    else if constexpr (OP == OP_SWEEP_RESID)
                        acc += vv[q] * (o1[q] + omega * o2[q] * o3[q]);
                    else
                        acc += vv[q] * o1[q];
                }
                done = true;
            }
        }
    }
    if (act && !done) {
        const int e1 = rp[i + 1];
        for (int e = rp[i] + sub; e < e1; e += G) {
            const int j = ci[e];
            if constexpr (OP == OP_PRESMOOTH)
                acc += v[e] * (omega * dinv[j] * b[j]);
            else if constexpr (OP == OP_SWEEP_RESID)
                acc += v[e] * (xin[j] + omega * dinv[j] * xs[j]);
            else
                acc += v[e] * xs[j];
        }
    }
    if constexpr (G > 1) {
#pragma unroll
        for (int d = G / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, G);
    }
    if (!act || sub != 0) return;
    if constexpr (OP == OP_SPMV) {
        xout[i] = acc;
    } else if constexpr (OP == OP_RESIDUAL) {
        rout[i] = b[i] - acc;
    } else if constexpr (OP == OP_SMOOTH) {
        xout[i] = xin[i] + omega * dinv[i] * (b[i] - acc);
    } else if constexpr (OP == OP_PRESMOOTH) {
        const T bi = b[i];
        xout[i] = omega * dinv[i] * bi;
        rout[i] = bi - acc;
    } else if constexpr (OP == OP_SWEEP_RESID) {
        xout[i] = xin[i] + omega * dinv[i] * xs[i];
        rout[i] = b[i] - acc;
    } else {
        xout[i] = xin[i] + acc;
    }
}

// lanes per row from the average row length
static inline int lanes_for(int n, int nnz) {
    const int avg = n > 0 ? nnz / n : 0;
    if (avg <= 6) return 1;
    if (avg <= 12) return 4;
    if (avg <= 24) return 8;
    if (avg <= 48) return 16;
    if (avg <= 96) return 32;
    return 64;
}

template <class T, int OP>
static void csr_op(int n, int nnz, const int *rp, const int *ci, const T *v, const T *xs, const T *dinv, T omega,
                   const T *b, const T *xin, T *xout, T *rout, hipStream_t st) {
    if (n == 0) return;
    const int G = lanes_for(n, nnz);
    const int blocks = nblocks((long)n * G, 256);
#define CASE(GG)                                                                                               \
    case GG:                                                                                                   \
        hipLaunchKernelGGL((k_csr_op<T, GG, OP>), dim3(blocks), dim3(256), 0, st, n, rp, ci, v, xs, dinv, omega, \
                           b, xin, xout, rout);                                                                \
        break;
    switch (G) { CASE(1) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64) }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

// The fine level of a scalar stage whose pattern is the 5-point stencil of an
// nx-wide grid, stored as five coefficient planes ell[k*n + i] for the
// columns i - nx, i - 1, i, i + 1, i + nx (k = 0..4; zero where row i has no
// such entry): the level's sweeps read them coalesced and need no row
// pointers or column indices.  The row sum takes the five terms in column
// order, as the CSR row loop takes a row's (ascending) entries, and a missing
// entry adds an exact zero, so the results are those of k_csr_op.
template <class T>
__global__ void k_ell5_fill(int n, int nx, const int *__restrict__ rp, const int *__restrict__ ci,
                            const T *__restrict__ v, T *__restrict__ ell) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T c[5] = {0, 0, 0, 0, 0};
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int d = ci[e] - i;   // one of -nx, -1, 0, 1, nx (checked at setup)
        const int k = (d == -nx) ? 0 : (d == -1) ? 1 : (d == 0) ? 2 : (d == 1) ? 3 : 4;
        c[k] = v[e];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) ell[(size_t)k * n + i] = c[k];
}

template <class T>
void vc_ell5_fill(int n, int nx, const int *rp, const int *ci, const T *v, T *ell, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_ell5_fill<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, nx, rp, ci, v, ell);
    CPTR_CHECK_LAUNCH();
}

// OP_PRESMOOTH, OP_SWEEP_RESID and OP_SMOOTH on the five planes (FP32 or FP64) (operands as
// in k_csr_op; a missing entry's column is clamped into range and its zero
// coefficient multiplies a finite value)
template <class T, int OP>
__global__ void __launch_bounds__(256) k_ell5_op(int n, int nx, const T *__restrict__ ell, const T *__restrict__ xs,
                                                 const T *__restrict__ dinv, T omega, const T *__restrict__ b,
                                                 const T *xin, T *xout, T *__restrict__ rout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int off[5] = {-nx, -1, 0, 1, nx};
    T vv[5], o1[5], o2[5], o3[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const int jr = i + off[q];
        const int j = jr < 0 ? 0 : (jr >= n ? n - 1 : jr);
        vv[q] = ell[(size_t)q * n + i];
        if constexpr (OP == OP_PRESMOOTH) {
            o1[q] = dinv[j];
            o2[q] = b[j];
        } else if constexpr (OP == OP_SWEEP_RESID) {
            o1[q] = xin[j];
            o2[q] = dinv[j];
            o3[q] = xs[j];
        } else {
            o1[q] = xs[j];
        }
    }
    T acc = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if constexpr (OP == OP_PRESMOOTH)
            acc += vv[q] * (omega * o1[q] * o2[q]);
        else if constexpr (OP == OP_SWEEP_RESID)
            acc += vv[q] * (o1[q] + omega * o2[q] * o3[q]);
        else
            acc += vv[q] * o1[q];
    }
    if constexpr (OP == OP_SMOOTH) {
        xout[i] = xin[i] + omega * dinv[i] * (b[i] - acc);
    } else if constexpr (OP == OP_PRESMOOTH) {
        const T bi = b[i];
        xout[i] = omega * dinv[i] * bi;
        rout[i] = bi - acc;
    } else {
        xout[i] = xin[i] + omega * dinv[i] * xs[i];
        rout[i] = b[i] - acc;
    }
}

template <class T, int OP>
static void ell5_op(int n, int nx, const T *ell, const T *xs, const T *dinv, T omega, const T *b, const T *xin,
                    T *xout, T *rout, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_ell5_op<T, OP>), dim3(nblocks(n, 256)), dim3(256), 0, st, n, nx, ell, xs, dinv, omega, b, xin,
                       xout, rout);
    CPTR_CHECK_LAUNCH();
}

template <class T>
void vc_ell5_presmooth_residual(int n, int nx, const T *ell, const T *dinv, T omega, const T *b, T *x, T *r,
                                hipStream_t st) {
    ell5_op<T, OP_PRESMOOTH>(n, nx, ell, nullptr, dinv, omega, b, nullptr, x, r, st);
}

template <class T>
void vc_ell5_sweep_residual(int n, int nx, const T *ell, const T *dinv, T omega, const T *b, const T *x, const T *r,
                            T *xout, T *rout, hipStream_t st) {
    ell5_op<T, OP_SWEEP_RESID>(n, nx, ell, r, dinv, omega, b, x, xout, rout, st);
}

template <class T>
void vc_ell5_smooth(int n, int nx, const T *ell, const T *dinv, T omega, const T *b, const T *xin, T *xout,
                    hipStream_t st) {
    ell5_op<T, OP_SMOOTH>(n, nx, ell, xin, dinv, omega, b, xin, xout, nullptr, st);
}

#define INST_ELL5(T)                                                                                              \
    template void vc_ell5_fill<T>(int, int, const int *, const int *, const T *, T *, hipStream_t);               \
    template void vc_ell5_presmooth_residual<T>(int, int, const T *, const T *, T, const T *, T *, T *, hipStream_t); \
    template void vc_ell5_sweep_residual<T>(int, int, const T *, const T *, T, const T *, const T *, const T *, T *, \
                                            T *, hipStream_t);                                                    \
    template void vc_ell5_smooth<T>(int, int, const T *, const T *, T, const T *, const T *, T *, hipStream_t);
INST_ELL5(float)
INST_ELL5(double)
#undef INST_ELL5

// first Jacobi sweep from a zero guess fused with the residual:
//   x_i = omega dinv_i b_i,   r_i = b_i - sum_j a_ij (omega dinv_j b_j)
template <class T>
void vc_presmooth_residual(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T omega,
                           const T *b, T *x, T *r, hipStream_t st) {
    csr_op<T, OP_PRESMOOTH>(n, nnz, rp, ci, v, nullptr, dinv, omega, b, nullptr, x, r, st);
}

// a further Jacobi sweep from x (with its residual r) fused with the new
// residual: xout = x + omega dinv r, rout = b - A xout (xout, rout distinct
// from x, r)
template <class T>
void vc_sweep_residual(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T omega,
                       const T *b, const T *x, const T *r, T *xout, T *rout, hipStream_t st) {
    csr_op<T, OP_SWEEP_RESID>(n, nnz, rp, ci, v, r, dinv, omega, b, x, xout, rout, st);
}

// y = A x
template <class T>
void vc_spmv(int n, int nnz, const int *rp, const int *ci, const T *v, const T *x, T *y, hipStream_t st) {
    csr_op<T, OP_SPMV>(n, nnz, rp, ci, v, x, nullptr, (T)0, nullptr, nullptr, y, nullptr, st);
}

// x = x + P xc
template <class T>
void vc_prolong_add(int n, int nnz, const int *rp, const int *ci, const T *v, const T *xc, T *x, hipStream_t st) {
    csr_op<T, OP_PROLONG>(n, nnz, rp, ci, v, xc, nullptr, (T)0, nullptr, x, x, nullptr, st);
}

// xout = xin + P xc
template <class T>
void vc_prolong_to(int n, int nnz, const int *rp, const int *ci, const T *v, const T *xc, const T *xin, T *xout,
                   hipStream_t st) {
    csr_op<T, OP_PROLONG>(n, nnz, rp, ci, v, xc, nullptr, (T)0, nullptr, xin, xout, nullptr, st);
}

// one damped Jacobi sweep: xout = xin + omega dinv (b - A xin)
template <class T>
void vc_smooth(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T omega, const T *b,
               const T *xin, T *xout, hipStream_t st) {
    csr_op<T, OP_SMOOTH>(n, nnz, rp, ci, v, xin, dinv, omega, b, xin, xout, nullptr, st);
}

// r = b - A x
template <class T>
void vc_residual(int n, int nnz, const int *rp, const int *ci, const T *v, const T *b, const T *x, T *r,
                 hipStream_t st) {
    csr_op<T, OP_RESIDUAL>(n, nnz, rp, ci, v, x, nullptr, (T)0, b, nullptr, nullptr, r, st);
}

// Chebyshev smoothing: the Chebyshev iteration on D^{-1} A over an interval
// [lmin, lmax] of its spectrum (three-term recurrence; theta and delta the
// interval's centre and half-width):
//   start  r = D^{-1} (b - A x),  d = r / theta   (x = 0: r = D^{-1} b, x set to 0)
//   step   x += d,  r -= D^{-1} A d,  d' = c1 d + c2 r
// with c1 = rho' rho, c2 = 2 rho' / delta and rho' = 1 / (2 theta / delta - rho)
// from rho = delta / theta, computed by the caller.  G lanes per row as above.
template <class T, int G, bool INIT>
__global__ void __launch_bounds__(256) k_cheb(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                              const T *__restrict__ v, const T *__restrict__ dinv,
                                              const T *__restrict__ b, const T *xs, T *x, T *r, T *dout, T theta,
                                              T c1, T c2) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / G), sub = (int)(t % G);
    const bool act = i < n;
    T acc = 0;
    if (act && xs) {
        const int e1 = rp[i + 1];
        for (int e = rp[i] + sub; e < e1; e += G) acc += v[e] * xs[ci[e]];
    }
    if constexpr (G > 1) {
#pragma unroll
        for (int d = G / 2; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, G);
    }
    if (!act || sub != 0) return;
    if constexpr (INIT) {
        const T ri = (b[i] - acc) * dinv[i];
        r[i] = ri;
        dout[i] = ri / theta;
        if (!xs) x[i] = (T)0;
    } else {
        const T di = xs[i];
        x[i] = x[i] + di;
        const T ri = r[i] - acc * dinv[i];
        r[i] = ri;
        dout[i] = c1 * di + c2 * ri;
    }
}

template <class T, bool INIT>
static void cheb_launch(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, const T *b,
                        const T *xs, T *x, T *r, T *dout, T theta, T c1, T c2, hipStream_t st) {
    if (n == 0) return;
    const int G = lanes_for(n, nnz);
    const int blocks = nblocks((long)n * G, 256);
#define CASE(GG)                                                                                               \
    case GG:                                                                                                   \
        hipLaunchKernelGGL((k_cheb<T, GG, INIT>), dim3(blocks), dim3(256), 0, st, n, rp, ci, v, dinv, b, xs, x, r, \
                           dout, theta, c1, c2);                                                               \
        break;
    switch (G) { CASE(1) CASE(4) CASE(8) CASE(16) CASE(32) CASE(64) }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

// start of a Chebyshev smoothing from x (x == nullptr: from zero, written to x0)
template <class T>
void vc_cheb_init(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, const T *b, const T *x,
                  T *x0, T *r, T *d, T theta, hipStream_t st) {
    cheb_launch<T, true>(n, nnz, rp, ci, v, dinv, b, x, x0, r, d, theta, (T)0, (T)0, st);
}

// one Chebyshev step: x += din, r -= D^{-1} A din, dout = c1 din + c2 r
template <class T>
void vc_cheb_step(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, const T *din, T *x, T *r,
                  T *dout, T c1, T c2, hipStream_t st) {
    cheb_launch<T, false>(n, nnz, rp, ci, v, dinv, nullptr, din, x, r, dout, (T)1, c1, c2, st);
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

// Algorithm 2 glue: out_i = r[i*b + comp] - sum_e cpl[e] * xs[ci[e]]
// (z_P = r_P - Abar[P,T] x_T when the T stage runs first; cpl holds the one
// coupling entry of every block that the update needs, contiguous)
template <class T>
__global__ void k_stage_input(int n, int b, const int *__restrict__ rp, const int *__restrict__ ci,
                              const T *__restrict__ cpl, int comp, const double *__restrict__ r,
                              const T *__restrict__ xs, T *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    T acc = (T)r[(size_t)i * b + comp];
    if (xs)
        for (int e = rp[i]; e < rp[i + 1]; ++e) acc -= cpl[e] * xs[ci[e]];
    out[i] = acc;
}

template <class T>
void ms_stage_input(int n, int b, const int *rp, const int *ci, const T *cpl, int comp, const double *r,
                    const T *xs, T *out, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_stage_input<T>, dim3(nblocks(n, 256)), dim3(256), 0, st, n, b, rp, ci, cpl, comp, r, xs,
                       out);
    CPTR_CHECK_LAUNCH();
}

// cpl[e] = slab[e*b + comp] (and its FP32 copy)
__global__ void k_gather_comp(int nnzb, int b, const double *__restrict__ slab, int comp, double *__restrict__ out,
                              float *__restrict__ out32) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnzb) return;
    const double v = slab[(size_t)e * b + comp];
    out[e] = v;
    if (out32) out32[e] = (float)v;
}

void ms_gather_comp(int nnzb, int b, const double *slab, int comp, double *out, float *out32, hipStream_t st) {
    if (nnzb == 0) return;
    hipLaunchKernelGGL(k_gather_comp, dim3(nblocks(nnzb, 256)), dim3(256), 0, st, nnzb, b, slab, comp, out, out32);
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

// the convergence-factor measurement of an FP32 V-cycle: y = A x in FP64,
// rounded to FP32 (the V-cycle's input), and e -= x with x from the V-cycle
__global__ void k_spmv_to_float(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                const double *__restrict__ v, const double *__restrict__ x, float *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) acc += v[e] * x[ci[e]];
    y[i] = (float)acc;
}

__global__ void k_sub_float(int n, const float *__restrict__ x, double *__restrict__ e) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) e[i] -= (double)x[i];
}

void vc_spmv_to_float(int n, const int *rp, const int *ci, const double *v, const double *x, float *y,
                      hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_spmv_to_float, dim3(nblocks(n, 256)), dim3(256), 0, st, n, rp, ci, v, x, y);
    CPTR_CHECK_LAUNCH();
}

void vc_sub_float(int n, const float *x, double *e, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_sub_float, dim3(nblocks(n, 256)), dim3(256), 0, st, n, x, e);
    CPTR_CHECK_LAUNCH();
}

#define INST(T)                                                                                                   \
    template void vc_presmooth_residual<T>(int, int, const int *, const int *, const T *, const T *, T, const T *, \
                                           T *, T *, hipStream_t);                                               \
    template void vc_spmv<T>(int, int, const int *, const int *, const T *, const T *, T *, hipStream_t);        \
    template void vc_sweep_residual<T>(int, int, const int *, const int *, const T *, const T *, T, const T *,   \
                                       const T *, const T *, T *, T *, hipStream_t);                            \
    template void vc_prolong_add<T>(int, int, const int *, const int *, const T *, const T *, T *, hipStream_t); \
    template void vc_cheb_init<T>(int, int, const int *, const int *, const T *, const T *, const T *, const T *,  \
                                  T *, T *, T *, T, hipStream_t);                                                  \
    template void vc_cheb_step<T>(int, int, const int *, const int *, const T *, const T *, const T *, T *, T *,   \
                                  T *, T, T, hipStream_t);                                                         \
    template void vc_prolong_to<T>(int, int, const int *, const int *, const T *, const T *, const T *, T *,     \
                                   hipStream_t);                                                                 \
    template void vc_smooth<T>(int, int, const int *, const int *, const T *, const T *, T, const T *, const T *, \
                               T *, hipStream_t);                                                                \
    template void vc_residual<T>(int, int, const int *, const int *, const T *, const T *, const T *, T *,       \
                                 hipStream_t);                                                                   \
    template void vc_dense_apply<T>(int, const T *, const T *, T *, hipStream_t);                                \
    template void ms_stage_input<T>(int, int, const int *, const int *, const T *, int, const double *,          \
                                    const T *, T *, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace cptr
