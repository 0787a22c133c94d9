// Outer operator apply (BSR SpMV) and the Arnoldi / Givens kernels of
// right-preconditioned restarted GMRES and flexible GMRES (the Krylov solver
// the paper applies to the left-scaled system, Eq. splitPrec2).
#include "internal.h"

namespace cptr {

// ---------------------------------------------------------------------------
// BSR SpMV
// ---------------------------------------------------------------------------

// b = 8: one wavefront per SPMV_ROWS consecutive block rows, whose blocks
// form one contiguous range of the value stream (512 B per block).  Every
// load instruction covers two blocks: half h of the wavefront takes block
// e0 + 2u + h, and lane p of a half holds the entry pair (p/4, 2(p%4)),
// (p/4, 2(p%4)+1) of it in one 16-byte load, with the matching pair of x.
// All SPMV_PAIRS pair loads of a batch are issued before the first product
// (ten blocks: the two interior rows of the 5-point pattern in one batch);
// each product is added to the partial sum of the row its block belongs to,
// and the four lanes of a block row and the two halves are combined with
// xor shuffles.  The value stream is read once: non-temporal loads keep it
// from evicting x from the caches.
constexpr int SPMV_ROWS = 2;
constexpr int SPMV_PAIRS = 5;

typedef double v2d __attribute__((ext_vector_type(2)));

template <bool RESID>
__global__ void __launch_bounds__(256) k_bsr8(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                              const double *__restrict__ A, const double *__restrict__ x,
                                              const double *__restrict__ rhs, double *__restrict__ y) {
    constexpr int R = SPMV_ROWS, PAIRS = SPMV_PAIRS;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int row0 = w * R;
    if (row0 >= n) return;
    const int nr = min(R, n - row0);
    const int h = lane >> 5, p = lane & 31;
    const int r = p >> 2, c0 = (p & 3) * 2;
    int rb[R + 1];
#pragma unroll
    for (int k = 0; k <= R; ++k) rb[k] = rp[row0 + min(k, nr)];
    const int ea = rb[0], eb = rb[R];
    double acc[R];
#pragma unroll
    for (int k = 0; k < R; ++k) acc[k] = 0.0;
    for (int e0 = ea; e0 < eb; e0 += 2 * PAIRS) {
        // clamped entry indices: every load is in bounds; entries past the
        // range are loaded again and not summed (every row holds its
        // diagonal block, so eb > ea)
        int ek[PAIRS], jk[PAIRS];
#pragma unroll
        for (int u = 0; u < PAIRS; ++u) {
            ek[u] = min(e0 + 2 * u + h, eb - 1);
            jk[u] = ci[ek[u]];
        }
        v2d av[PAIRS], xv[PAIRS];
#pragma unroll
        for (int u = 0; u < PAIRS; ++u) {
            av[u] = __builtin_nontemporal_load((const v2d *)(A + (size_t)ek[u] * 64 + r * 8 + c0));
            xv[u] = *(const v2d *)(x + (size_t)jk[u] * 8 + c0);
        }
#pragma unroll
        for (int u = 0; u < PAIRS; ++u) {
            const int e = e0 + 2 * u + h;
            if (e < eb) {
                const double pr = av[u].x * xv[u].x + av[u].y * xv[u].y;
#pragma unroll
                for (int k = 0; k < R; ++k)
                    if (e >= rb[k] && e < rb[k + 1]) acc[k] += pr;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        double v = acc[k];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 32, 64);
        if (k < nr && lane < 32 && (p & 3) == 0) {
            const size_t o = (size_t)(row0 + k) * 8 + r;
            y[o] = RESID ? rhs[o] - v : v;
        }
    }
}

// generic b: one thread per scalar row (i, r)
template <bool RESID>
__global__ void k_bsr_gen(int n, int b, const int *__restrict__ rp, const int *__restrict__ ci,
                          const double *__restrict__ A, const double *__restrict__ x,
                          const double *__restrict__ rhs, double *__restrict__ y) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)n * b) return;
    const int i = (int)(t / b), r = (int)(t % b);
    double acc = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const double *Bk = A + (size_t)e * b * b + r * b;
        const double *xc = x + (size_t)ci[e] * b;
        for (int c = 0; c < b; ++c) acc += Bk[c] * xc[c];
    }
    y[t] = RESID ? rhs[t] - acc : acc;
}

void launch_bsr_spmv(int n, int b, const int *rp, const int *ci, const double *A, const double *x, double *y,
                     hipStream_t s) {
    if (n == 0) return;
    if (b == 8)
        hipLaunchKernelGGL(k_bsr8<false>, dim3((n + SPMV_ROWS * 4 - 1) / (SPMV_ROWS * 4)), dim3(256), 0, s, n, rp,
                           ci, A, x, nullptr, y);
    else
        hipLaunchKernelGGL(k_bsr_gen<false>, dim3(((long)n * b + 255) / 256), dim3(256), 0, s, n, b, rp, ci, A, x,
                           nullptr, y);
    CPTR_CHECK_LAUNCH();
}

void launch_bsr_residual(int n, int b, const int *rp, const int *ci, const double *A, const double *x,
                         const double *rhs, double *r, hipStream_t s) {
    if (n == 0) return;
    if (b == 8)
        hipLaunchKernelGGL(k_bsr8<true>, dim3((n + SPMV_ROWS * 4 - 1) / (SPMV_ROWS * 4)), dim3(256), 0, s, n, rp,
                           ci, A, x, rhs, r);
    else
        hipLaunchKernelGGL(k_bsr_gen<true>, dim3(((long)n * b + 255) / 256), dim3(256), 0, s, n, b, rp, ci, A, x,
                           rhs, r);
    CPTR_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// reductions: per-block partials in a fixed order, then one block sums them
// in a fixed order -> deterministic results (no floating-point atomics)
// ---------------------------------------------------------------------------
constexpr int KR_THREADS = 256;
constexpr int KR_GROUP = 8;   // vectors handled per pass of the multi-dot

int kr_nblk(int N) {
    long b = ((long)N + KR_THREADS * 8 - 1) / (KR_THREADS * 8);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

__device__ inline double block_sum(double v, double *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w];
    return s;   // valid in thread 0
}

// partial[blk*(k+1) + j] = sum over the block's rows of V_j . w (j < k), and
// partial[blk*(k+1) + k] = w . w
__global__ void __launch_bounds__(KR_THREADS) k_mdot(int N, int k, const double *__restrict__ V, size_t ldv,
                                                     const double *__restrict__ w, double *__restrict__ partial) {
    __shared__ double red[KR_GROUP][KR_THREADS / 64];
    const long chunk = ((long)N + gridDim.x - 1) / gridDim.x;
    const long r0 = (long)blockIdx.x * chunk;
    const long r1 = min((long)N, r0 + chunk);
    for (int j0 = 0; j0 <= k; j0 += KR_GROUP) {
        double acc[KR_GROUP];
#pragma unroll
        for (int q = 0; q < KR_GROUP; ++q) acc[q] = 0.0;
        // four rows per pass: their loads are all issued before the sums
        // (each accumulator still takes the thread's rows in ascending order)
        long r = r0 + threadIdx.x;
        for (; r + 3 * KR_THREADS < r1; r += 4 * KR_THREADS) {
            double wr[4], vr[KR_GROUP][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) wr[u] = w[r + u * KR_THREADS];
#pragma unroll
            for (int q = 0; q < KR_GROUP; ++q) {
                const int j = j0 + q;
#pragma unroll
                for (int u = 0; u < 4; ++u) vr[q][u] = (j < k) ? V[(size_t)j * ldv + r + u * KR_THREADS] : wr[u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int q = 0; q < KR_GROUP; ++q)
                    if (j0 + q <= k) acc[q] += vr[q][u] * wr[u];
            }
        }
        for (; r < r1; r += KR_THREADS) {
            const double wr = w[r];
#pragma unroll
            for (int q = 0; q < KR_GROUP; ++q) {
                const int j = j0 + q;
                if (j < k) acc[q] += V[(size_t)j * ldv + r] * wr;
                else if (j == k) acc[q] += wr * wr;
            }
        }
        // the group's block sums together (same order as block_sum: a
        // shuffle tree per wavefront, then the wavefronts in order)
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int q = 0; q < KR_GROUP; ++q)
            for (int d = 32; d >= 1; d >>= 1) acc[q] += __shfl_xor(acc[q], d, 64);
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < KR_GROUP; ++q) red[q][wave] = acc[q];
        }
        __syncthreads();
        if ((int)threadIdx.x < KR_GROUP && j0 + (int)threadIdx.x <= k) {
            const int q = threadIdx.x;
            double sum = 0.0;
            for (int w = 0; w < KR_THREADS / 64; ++w) sum += red[q][w];
            partial[(size_t)blockIdx.x * (k + 1) + j0 + q] = sum;
        }
        __syncthreads();   // red is reused by the next group
    }
}

void kr_mdot(int N, int k, const double *V, size_t ldv, const double *w, double *partial, int nblk,
             hipStream_t st) {
    hipLaunchKernelGGL(k_mdot, dim3(nblk), dim3(KR_THREADS), 0, st, N, k, V, ldv, w, partial);
    CPTR_CHECK_LAUNCH();
}

// out[j] = sum over blocks of partial[blk*k + j]: one block per output, each
// thread sums a fixed strided subset, then a fixed-shape tree (deterministic)
__global__ void __launch_bounds__(256) k_reduce(const double *__restrict__ partial, int nblk, int k,
                                                double *__restrict__ out) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partial[(size_t)b * k + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}

void kr_reduce(const double *partial, int nblk, int k, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(k), dim3(256), 0, st, partial, nblk, k, out);
    CPTR_CHECK_LAUNCH();
}

// w -= sum_j h_j V_j (classical Gram-Schmidt projection), partial[blk] = |w|^2
__global__ void __launch_bounds__(KR_THREADS) k_update(int N, int k, const double *__restrict__ V, size_t ldv,
                                                       const double *__restrict__ h, double *__restrict__ w,
                                                       double *__restrict__ partial) {
    __shared__ double hs[256];
    __shared__ double lds[KR_THREADS / 64];
    for (int j = threadIdx.x; j < k; j += blockDim.x) hs[j] = h[j];
    __syncthreads();
    const long chunk = ((long)N + gridDim.x - 1) / gridDim.x;
    const long r0 = (long)blockIdx.x * chunk;
    const long r1 = min((long)N, r0 + chunk);
    double nrm = 0.0;
    // four rows per pass (their loads of each V_j issued together); every
    // row and the norm keep their order
    long r = r0 + threadIdx.x;
    for (; r + 3 * KR_THREADS < r1; r += 4 * KR_THREADS) {
        double acc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = w[r + u * KR_THREADS];
        for (int j = 0; j < k; ++j) {
            const double hj = hs[j];
            double vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) vv[u] = V[(size_t)j * ldv + r + u * KR_THREADS];
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] -= hj * vv[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            w[r + u * KR_THREADS] = acc[u];
            nrm += acc[u] * acc[u];
        }
    }
    for (; r < r1; r += KR_THREADS) {
        double acc = w[r];
        for (int j = 0; j < k; ++j) acc -= hs[j] * V[(size_t)j * ldv + r];
        w[r] = acc;
        nrm += acc * acc;
    }
    double s = block_sum(nrm, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void kr_update(int N, int k, const double *V, size_t ldv, const double *h, double *w, double *partial, int nblk,
               hipStream_t st) {
    if (k > 256) throw Error(CPTR_E_ARG, "restart too long");
    hipLaunchKernelGGL(k_update, dim3(nblk), dim3(KR_THREADS), 0, st, N, k, V, ldv, h, w, partial);
    CPTR_CHECK_LAUNCH();
}

__global__ void __launch_bounds__(KR_THREADS) k_norm2(int N, const double *__restrict__ x,
                                                      double *__restrict__ partial) {
    __shared__ double lds[KR_THREADS / 64];
    const long chunk = ((long)N + gridDim.x - 1) / gridDim.x;
    const long r0 = (long)blockIdx.x * chunk;
    const long r1 = min((long)N, r0 + chunk);
    double nrm = 0.0;
    for (long r = r0 + threadIdx.x; r < r1; r += KR_THREADS) nrm += x[r] * x[r];
    double s = block_sum(nrm, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

void kr_norm2_partial(int N, const double *x, double *partial, int nblk, hipStream_t st) {
    hipLaunchKernelGGL(k_norm2, dim3(nblk), dim3(KR_THREADS), 0, st, N, x, partial);
    CPTR_CHECK_LAUNCH();
}

// Arnoldi step j finishes on one block: sum the |w|^2 partials (fixed order),
// store column j of H (h_{i,j} from hcol, plus a second-pass correction when
// re-orthogonalised), h_{j+1,j} = |w|; apply the previous Givens rotations,
// form the new one, update g.  scal[0] = 1 / h_{j+1,j} for the normalisation.
// hostinfo (host-visible): [ |g_{j+1}|, h_{j+1,j}, |A z_j| ].
// H is column-major with leading dimension m+1.
__global__ void k_arnoldi_finish(int j, int m, double *H, double *cs, double *sn, double *g,
                                 const double *hcol, const double *hcol2, const double *nrm_partial, int nblk,
                                 double *scal, double *hostinfo) {
    double p = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) p += nrm_partial[b];
    // fixed-shape tree over the block
    __shared__ double red[256];
    red[threadIdx.x] = p;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const int ld = m + 1;
    double *Hc = H + (size_t)j * ld;
    for (int i = 0; i <= j; ++i) Hc[i] = hcol[i] + (hcol2 ? hcol2[i] : 0.0);
    const double wn = sqrt(red[0]);
    const double wnorm0 = sqrt(hcol[j + 1]);   // |A z_j| from the first multi-dot
    Hc[j + 1] = wn;
    for (int i = 0; i < j; ++i) {
        double t = cs[i] * Hc[i] + sn[i] * Hc[i + 1];
        Hc[i + 1] = -sn[i] * Hc[i] + cs[i] * Hc[i + 1];
        Hc[i] = t;
    }
    const double den = hypot(Hc[j], Hc[j + 1]);
    cs[j] = Hc[j] / den;
    sn[j] = Hc[j + 1] / den;
    const double hj1 = Hc[j + 1];
    Hc[j] = den;
    Hc[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    scal[0] = (hj1 != 0.0) ? 1.0 / hj1 : 0.0;
    hostinfo[0] = fabs(g[j + 1]);
    hostinfo[1] = hj1;
    hostinfo[2] = wnorm0;
}

void kr_arnoldi_finish2(int j, int m, double *H, double *cs, double *sn, double *g, const double *hcol,
                        const double *hcol2, const double *nrm_partial, int nblk, double *scal, double *hostinfo,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_arnoldi_finish, dim3(1), dim3(256), 0, st, j, m, H, cs, sn, g, hcol, hcol2, nrm_partial,
                       nblk, scal, hostinfo);
    CPTR_CHECK_LAUNCH();
}

__global__ void k_scale(int N, const double *__restrict__ w, const double *__restrict__ scal,
                        double *__restrict__ v) {
    const double s = scal[0];
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long st = (long)gridDim.x * blockDim.x;
    for (; i < N; i += st) v[i] = w[i] * s;
}

void kr_scale(int N, const double *w, const double *scal, double *v, hipStream_t st) {
    long g = ((long)N + 255) / 256;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_scale, dim3((int)g), dim3(256), 0, st, N, w, scal, v);
    CPTR_CHECK_LAUNCH();
}

// start of a restart cycle from the residual r: beta = |r| (partials summed in
// a fixed order), v0 = r / beta, g = beta e_1.  hostinfo[0] = beta.
__global__ void k_cycle_prep(const double *nrm_partial, int nblk, int m, double *g, double *scal,
                             double *hostinfo) {
    __shared__ double red[256];
    double p = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) p += nrm_partial[b];
    red[threadIdx.x] = p;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double beta = sqrt(red[0]);
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        scal[0] = (beta != 0.0) ? 1.0 / beta : 0.0;
        hostinfo[0] = beta;
    }
}

void kr_cycle_prep(const double *nrm_partial, int nblk, int m, double *g, double *scal, double *hostinfo,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_cycle_prep, dim3(1), dim3(256), 0, st, nrm_partial, nblk, m, g, scal, hostinfo);
    CPTR_CHECK_LAUNCH();
}

// y = R^{-1} g for the k x k upper triangle of the rotated H (back substitution)
__global__ void k_solve_upper(int k, int m, const double *H, const double *g, double *y) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int ld = m + 1;
    for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int c = i + 1; c < k; ++c) t -= H[(size_t)c * ld + i] * y[c];
        y[i] = t / H[(size_t)i * ld + i];
    }
}

void kr_solve_upper(int k, int m, const double *H, const double *g, double *y, hipStream_t st) {
    hipLaunchKernelGGL(k_solve_upper, dim3(1), dim3(64), 0, st, k, m, H, g, y);
    CPTR_CHECK_LAUNCH();
}

// x += sum_j y_j Z_j
template <class TZ>
__global__ void k_combine(int N, int k, const TZ *__restrict__ Z, size_t ldz, const double *__restrict__ y,
                          double *__restrict__ x) {
    __shared__ double ys[256];
    for (int j = threadIdx.x; j < k; j += blockDim.x) ys[j] = y[j];
    __syncthreads();
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    long st = (long)gridDim.x * blockDim.x;
    for (; i < N; i += st) {
        double acc = x[i];
        for (int j = 0; j < k; ++j) acc += ys[j] * (double)Z[(size_t)j * ldz + i];
        x[i] = acc;
    }
}

template <class TZ>
void kr_combine(int N, int k, const TZ *Z, size_t ldz, const double *y, double *x, hipStream_t st) {
    if (k > 256) throw Error(CPTR_E_ARG, "restart too long");
    long g = ((long)N + 255) / 256;
    if (g > 16384) g = 16384;
    hipLaunchKernelGGL(k_combine<TZ>, dim3((int)g), dim3(256), 0, st, N, k, Z, ldz, y, x);
    CPTR_CHECK_LAUNCH();
}
template void kr_combine<double>(int, int, const double *, size_t, const double *, double *, hipStream_t);
template void kr_combine<float>(int, int, const float *, size_t, const double *, double *, hipStream_t);

}  // namespace cptr
