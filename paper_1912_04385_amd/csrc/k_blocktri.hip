// Exact sub-solves beyond the dense limit (the Schur-complement quality study
// of Sec. "Numerical Results", whose direct solves with B_PP, C_TT and B_ee
// reach 160 x 160 grids).  On a 5-point grid the operators are block
// tridiagonal by grid rows: with the rows ordered group by group (group y =
// the unknowns of grid row y: g = nx rows for a scalar operator, g = 2 nx for
// the two unknowns of B_ee), A = tridiag(L_y, D_y, U_y), and the block LU
// factorisation
//   S_0 = D_0,   S_y = D_y - L_y G_{y-1},   G_y = S_y^{-1} U_y
// gives the exact solve
//   z_y = S_y^{-1} (b_y - L_y z_{y-1})        (y ascending)
//   x_y = z_y - G_y x_{y+1}                    (y descending).
// S_y^{-1} comes from the dense Gauss-Jordan inverse with partial pivoting;
// the couplings L_y, U_y stay sparse (read from the operator's rows and from
// its transpose).  perm[r] is the group-major position y g + p of operator
// row r, rowof its inverse.
#include "internal.h"

namespace cptr {

constexpr int BT_THREADS = 256;
constexpr int BT_WAVES = BT_THREADS / 64;

// flag |= 1 when an entry couples groups more than one apart
__global__ void k_bt_check(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                           const int *__restrict__ perm, int g, int *flag) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int yr = perm[r] / g;
    for (int e = rp[r]; e < rp[r + 1]; ++e) {
        const int yc = perm[ci[e]] / g;
        if (yc - yr > 1 || yr - yc > 1) atomicOr(flag, 1);
    }
}

// dense g x g pattern as CSR indices (the input form of the dense inverse)
__global__ void k_bt_dense_index(int g, int *__restrict__ drp, int *__restrict__ dci) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= g) drp[t] = (int)(t * g);
    if (t < (long)g * g) dci[t] = (int)(t % g);
}

// S_y[p][:] = D_y[p][:] - sum over the row's entries into group y-1 of
// a_rc G_{y-1}[pos(c)][:]; one workgroup per row p of the group
__global__ void __launch_bounds__(BT_THREADS) k_bt_schur(int y, int g, const int *__restrict__ rp,
                                                          const int *__restrict__ ci, const double *__restrict__ v,
                                                          const int *__restrict__ perm, const int *__restrict__ rowof,
                                                          const double *__restrict__ Gprev, double *__restrict__ S) {
    __shared__ double row[BT_MAX_GROUP];
    const int p = blockIdx.x;
    const int r = rowof[(size_t)y * g + p];
    const int e0 = rp[r], e1 = rp[r + 1];
    for (int j = threadIdx.x; j < g; j += BT_THREADS) row[j] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int e = e0; e < e1; ++e) {
            const int q = perm[ci[e]];
            if (q / g == y) row[q % g] = v[e];
        }
    __syncthreads();
    for (int j = threadIdx.x; j < g; j += BT_THREADS) {
        double s = row[j];
        if (Gprev)
            for (int e = e0; e < e1; ++e) {
                const int q = perm[ci[e]];
                if (q / g == y - 1) s -= v[e] * Gprev[(size_t)(q % g) * g + j];
            }
        S[(size_t)p * g + j] = s;
    }
}

// G_y[i][p] = sum over the entries (r, a) of column c = rowof[(y+1) g + p]
// with r in group y of Sinv_y[i][pos(r)] a (the transpose lists column c's
// entries); one workgroup per row i
__global__ void __launch_bounds__(BT_THREADS) k_bt_g(int y, int g, const int *__restrict__ atrp,
                                                      const int *__restrict__ atci, const double *__restrict__ atv,
                                                      const int *__restrict__ perm, const int *__restrict__ rowof,
                                                      const double *__restrict__ Sinv, double *__restrict__ G) {
    const int i = blockIdx.x;
    for (int p = threadIdx.x; p < g; p += BT_THREADS) {
        const int c = rowof[(size_t)(y + 1) * g + p];
        double s = 0.0;
        for (int f = atrp[c]; f < atrp[c + 1]; ++f) {
            const int q = perm[atci[f]];
            if (q / g == y) s += Sinv[(size_t)i * g + q % g] * atv[f];
        }
        G[(size_t)i * g + p] = s;
    }
}

__device__ inline double bt_wave_sum(double a) {
    for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o, 64);
    return a;
}

// forward step y: t = b_y - L_y z_{y-1} (every workgroup forms all of t in
// LDS), then z_y = Sinv_y t, one wavefront per row
template <class T>
__global__ void __launch_bounds__(BT_THREADS) k_bt_fwd(int y, int g, const int *__restrict__ rp,
                                                        const int *__restrict__ ci, const double *__restrict__ v,
                                                        const int *__restrict__ perm, const int *__restrict__ rowof,
                                                        const T *__restrict__ b, const double *__restrict__ Sinv,
                                                        double *__restrict__ z) {
    __shared__ double t[BT_MAX_GROUP];
    for (int p = threadIdx.x; p < g; p += BT_THREADS) {
        const int r = rowof[(size_t)y * g + p];
        double s = (double)b[r];
        if (y > 0)
            for (int e = rp[r]; e < rp[r + 1]; ++e) {
                const int q = perm[ci[e]];
                if (q / g == y - 1) s -= v[e] * z[q];
            }
        t[p] = s;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * BT_WAVES + (threadIdx.x >> 6);
    if (i >= g) return;
    const double *Si = Sinv + (size_t)i * g;
    double a = 0.0;
    for (int j = lane; j < g; j += 64) a += Si[j] * t[j];
    a = bt_wave_sum(a);
    if (lane == 0) z[(size_t)y * g + i] = a;
}

// backward step y: x_y = z_y - G_y x_{y+1} (no G on the last group), one
// wavefront per row; the result also goes to the caller's vector in operator
// order
template <class T>
__global__ void __launch_bounds__(BT_THREADS) k_bt_bwd(int y, int g, const double *__restrict__ G,
                                                        const double *__restrict__ z, double *__restrict__ xw,
                                                        const int *__restrict__ rowof, T *__restrict__ x) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * BT_WAVES + (threadIdx.x >> 6);
    if (i >= g) return;
    double a = 0.0;
    if (G) {
        const double *Gi = G + (size_t)i * g;
        const double *xn = xw + (size_t)(y + 1) * g;
        for (int j = lane; j < g; j += 64) a += Gi[j] * xn[j];
        a = bt_wave_sum(a);
    }
    if (lane == 0) {
        const size_t q = (size_t)y * g + i;
        const double val = z[q] - a;
        xw[q] = val;
        x[rowof[q]] = (T)val;
    }
}

void bt_check(int n, const int *rp, const int *ci, const int *perm, int g, int *flag, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_bt_check, dim3((n + 255) / 256), dim3(256), 0, s, n, rp, ci, perm, g, flag);
    CPTR_CHECK_LAUNCH();
}

void bt_dense_index(int g, int *drp, int *dci, hipStream_t s) {
    const long m = (long)g * g + 1;
    hipLaunchKernelGGL(k_bt_dense_index, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, g, drp, dci);
    CPTR_CHECK_LAUNCH();
}

void bt_schur(int y, int g, const int *rp, const int *ci, const double *v, const int *perm, const int *rowof,
              const double *Gprev, double *S, hipStream_t s) {
    hipLaunchKernelGGL(k_bt_schur, dim3(g), dim3(BT_THREADS), 0, s, y, g, rp, ci, v, perm, rowof, Gprev, S);
    CPTR_CHECK_LAUNCH();
}

void bt_g(int y, int g, const int *atrp, const int *atci, const double *atv, const int *perm, const int *rowof,
          const double *Sinv, double *G, hipStream_t s) {
    hipLaunchKernelGGL(k_bt_g, dim3(g), dim3(BT_THREADS), 0, s, y, g, atrp, atci, atv, perm, rowof, Sinv, G);
    CPTR_CHECK_LAUNCH();
}

template <class T>
void bt_solve(int ng, int g, const int *rp, const int *ci, const double *v, const int *perm, const int *rowof,
              const double *Sinv, const double *G, double *z, double *xw, const T *b, T *x, hipStream_t s) {
    const dim3 grid((g + BT_WAVES - 1) / BT_WAVES), block(BT_THREADS);
    const size_t gg = (size_t)g * g;
    for (int y = 0; y < ng; ++y)
        hipLaunchKernelGGL(k_bt_fwd<T>, grid, block, 0, s, y, g, rp, ci, v, perm, rowof, b, Sinv + y * gg, z);
    for (int y = ng - 1; y >= 0; --y)
        hipLaunchKernelGGL(k_bt_bwd<T>, grid, block, 0, s, y, g, (y + 1 < ng) ? G + y * gg : nullptr, z, xw, rowof,
                           x);
    CPTR_CHECK_LAUNCH();
}

template void bt_solve<double>(int, int, const int *, const int *, const double *, const int *, const int *,
                               const double *, const double *, double *, double *, const double *, double *,
                               hipStream_t);
template void bt_solve<float>(int, int, const int *, const int *, const double *, const int *, const int *,
                              const double *, const double *, double *, double *, const float *, float *,
                              hipStream_t);

}  // namespace cptr
