// Static condensation of the full Newton system (Sec. "Static-Condensation
// Strategy", Eqs. global and reduced): the secondary unknowns couple only
// within their cell, so J22 is block diagonal and J21 cell-local, and
//   Q_j = J22_jj^{-1} J21_jj,   q_j = J22_jj^{-1} r2_j              (per cell)
//   A_ij = J11_ij - J12_ij Q_j,   b_i = -r1_i + sum_j J12_ij q_j     (per block)
//   d2_j = -q_j - Q_j d1_j                                          (recovery)
// The reduced system keeps the pattern of J11.
#include "internal.h"

#include <algorithm>

namespace cptr {

// Per cell, one group of 8 lanes: lane r < n2 holds row r of the augmented
// block [J22_jj | J21_jj (8 columns, zero beyond n1) | r2_j] in registers.  Gauss-Jordan with partial
// pivoting without row exchanges (a row that served as pivot is marked), the
// pivot row broadcast by shuffles; the row that pivoted column k then holds
// row k of the solution, scaled by its pivot.  flag: lowest singular cell.
constexpr int CD_G = 8;

template <int N2>
__global__ void __launch_bounds__(256) k_condense_cells(int n, int n1, const double *__restrict__ J21,
                                                        const double *__restrict__ J22,
                                                        const double *__restrict__ r2, double *__restrict__ Q,
                                                        double *__restrict__ q, int *flag) {
    constexpr int NC = N2 + 9;   // J22 columns, 8 for J21, r2 last
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = (int)(t / CD_G), r = (int)(t % CD_G);
    const int gbase = (threadIdx.x & 63) - r;
    const bool act = j < n;
    const bool own = act && r < N2;
    double row[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) row[c] = 0.0;
    if (own) {
#pragma unroll
        for (int c = 0; c < N2; ++c) row[c] = J22[((size_t)j * N2 + r) * N2 + c];
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < n1) row[N2 + c] = J21[((size_t)j * N2 + r) * n1 + c];
        row[NC - 1] = r2[(size_t)j * N2 + r];
    }
    bool used = !own;
    int myk = -1;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < N2; ++k) {
        // pivot: the first unused row with the largest |row[k]|
        const double mine = used ? -1.0 : fabs(row[k]);
        double best = -2.0;
        int who = 0;
#pragma unroll
        for (int s = 0; s < N2; ++s) {
            const double o = __shfl(mine, gbase + s, 64);
            if (o > best) { best = o; who = s; }
        }
        if (best <= 0.0) bad = true;
        double prow[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) prow[c] = __shfl(row[c], gbase + who, 64);
        if (own && !bad) {
            if (r == who) {
                used = true;
                myk = k;
            } else {
                const double f = row[k] / prow[k];
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    if (c > k) row[c] -= f * prow[c];
                row[k] = 0.0;
            }
        }
    }
    if (!act) return;
    if (bad) {
        if (r == 0) atomicMin(flag, j);
        return;
    }
    if (own) {
        const double d = row[myk];
#pragma unroll
        for (int c = 0; c < 8; ++c)
            if (c < n1) Q[((size_t)j * N2 + myk) * n1 + c] = row[N2 + c] / d;
        q[(size_t)j * N2 + myk] = row[NC - 1] / d;
    }
}

// Per block row, one wavefront: lane (r, c) of the n1 x n1 block forms
// A_ij[r][c] = J11_ij[r][c] - sum_k J12_ij[r][k] Q_j[k][c] (k ascending) for
// every block of the row; lanes with c = 0 also sum b_i[r] over the row's
// blocks in order.  The blocks are taken CH at a time with all their
// operands loaded before the sums.
template <int N2>
__global__ void __launch_bounds__(64) k_condense_blocks(int n, int n1, const int *__restrict__ rp,
                                                        const int *__restrict__ ci, const double *__restrict__ J11,
                                                        const double *__restrict__ J12,
                                                        const double *__restrict__ Q, const double *__restrict__ q,
                                                        const double *__restrict__ r1, double *__restrict__ A,
                                                        double *__restrict__ b) {
    constexpr int CH = (N2 <= 2) ? 6 : (N2 <= 4 ? 4 : 2);
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    if (i >= n || lane >= n1 * n1) return;
    const int r = lane / n1, c = lane % n1;
    double acc = -r1[(size_t)i * n1 + r];
    const int e0 = rp[i], e1 = rp[i + 1];
    for (int base = e0; base < e1; base += CH) {
        int js[CH];
        double a[CH], x[CH][N2 > 0 ? N2 : 1], y[CH][N2 > 0 ? N2 : 1], z[CH][N2 > 0 ? N2 : 1];
#pragma unroll
        for (int u = 0; u < CH; ++u) js[u] = (base + u < e1) ? ci[base + u] : 0;
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const bool on = base + u < e1;
            const size_t e = (size_t)(base + u);
            a[u] = on ? J11[(e * n1 + r) * n1 + c] : 0.0;
#pragma unroll
            for (int k = 0; k < N2; ++k) {
                x[u][k] = on ? J12[(e * n1 + r) * N2 + k] : 0.0;
                y[u][k] = on ? Q[((size_t)js[u] * N2 + k) * n1 + c] : 0.0;
                z[u][k] = (on && c == 0) ? q[(size_t)js[u] * N2 + k] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            if (base + u >= e1) break;
            double v = a[u], t = 0.0;
#pragma unroll
            for (int k = 0; k < N2; ++k) {
                v -= x[u][k] * y[u][k];
                t += x[u][k] * z[u][k];
            }
            A[((size_t)(base + u) * n1 + r) * n1 + c] = v;
            acc += t;
        }
    }
    if (c == 0) b[(size_t)i * n1 + r] = acc;
}

// d2_j[k] = -q_j[k] - sum_c Q_j[k][c] d1_j[c], one thread per secondary unknown
__global__ void k_condense_recover(int n, int n1, int n2, const double *__restrict__ Q,
                                   const double *__restrict__ q, const double *__restrict__ d1,
                                   double *__restrict__ d2) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)n * n2) return;
    const int j = (int)(t / n2), k = (int)(t % n2);
    const double *Qk = Q + ((size_t)j * n2 + k) * n1;
    double s = -q[t];
    for (int c = 0; c < n1; ++c) s -= Qk[c] * d1[(size_t)j * n1 + c];
    d2[t] = s;
}

// Well elimination (remark closing Sec. "Static-Condensation Strategy"):
// well w, with nw unknowns, perforates one cell c_w and couples to its
// primary unknowns only, so
//   Qw_w = Jww_w^{-1} Jw1_w,  qw_w = Jww_w^{-1} rw_w                  (per well)
//   A_cc -= J1w_w Qw_w,  b_c += J1w_w qw_w   (diagonal block of c_w)
//   dw_w = -qw_w - Qw_w d1_c                                       (recovery)
// One workgroup: thread w factors well w (Gauss-Jordan with partial pivoting
// on [Jww | Jw1 | rw], NW <= 8 rows held in registers); then the wells update
// their cells' diagonal blocks one after the other in well order (wells that
// share a cell add their terms in that order), lane (r, c) of the block.
// flag[0]: lowest well with a singular Jww; flag[1]: lowest well whose cell
// has no stored diagonal block.
constexpr int WL_THREADS = 256;

template <int NW>
__global__ void __launch_bounds__(WL_THREADS) k_condense_wells(int nwells, int n1, const int *__restrict__ rp,
                                                               const int *__restrict__ ci,
                                                               const int *__restrict__ wcell,
                                                               const double *__restrict__ J1w,
                                                               const double *__restrict__ Jw1,
                                                               const double *__restrict__ Jww,
                                                               const double *__restrict__ rw, double *__restrict__ A,
                                                               double *__restrict__ b, double *__restrict__ Qw,
                                                               double *__restrict__ qw, int *flag) {
    constexpr int NC = NW + 9;     // Jww columns, 8 for Jw1, rw last
    __shared__ int s_bad[2];
    if (threadIdx.x == 0) { s_bad[0] = 0x7fffffff; s_bad[1] = 0x7fffffff; }
    __syncthreads();
    for (int w = threadIdx.x; w < nwells; w += WL_THREADS) {
        // the perforated cell's diagonal block must be stored
        const int cell = wcell[w];
        int e = rp[cell];
        while (e < rp[cell + 1] && ci[e] != cell) ++e;
        if (e == rp[cell + 1]) {
            atomicMin(&s_bad[1], w);
            atomicMin(flag + 1, w);
            continue;
        }
        double m[NW][NC];
#pragma unroll
        for (int r = 0; r < NW; ++r) {
#pragma unroll
            for (int c = 0; c < NW; ++c) m[r][c] = Jww[((size_t)w * NW + r) * NW + c];
#pragma unroll
            for (int c = 0; c < 8; ++c) m[r][NW + c] = (c < n1) ? Jw1[((size_t)w * NW + r) * n1 + c] : 0.0;
            m[r][NC - 1] = rw[(size_t)w * NW + r];
        }
        bool bad = false;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            int p = k;
            double best = fabs(m[k][k]);
#pragma unroll
            for (int r = k + 1; r < NW; ++r)
                if (fabs(m[r][k]) > best) { best = fabs(m[r][k]); p = r; }
            if (!(best > 0.0)) { bad = true; break; }
            if (p != k) {
#pragma unroll
                for (int r = k + 1; r < NW; ++r)
                    if (r == p) {
#pragma unroll
                        for (int c = 0; c < NC; ++c) { const double t = m[k][c]; m[k][c] = m[r][c]; m[r][c] = t; }
                    }
            }
            const double inv = 1.0 / m[k][k];
#pragma unroll
            for (int c = 0; c < NC; ++c) m[k][c] *= inv;
#pragma unroll
            for (int r = 0; r < NW; ++r) {
                if (r == k) continue;
                const double f = m[r][k];
#pragma unroll
                for (int c = 0; c < NC; ++c) m[r][c] -= f * m[k][c];
            }
        }
        if (bad) {
            atomicMin(&s_bad[0], w);
            atomicMin(flag, w);
            continue;
        }
#pragma unroll
        for (int r = 0; r < NW; ++r) {
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < n1) Qw[((size_t)w * NW + r) * n1 + c] = m[r][NW + c];
            qw[(size_t)w * NW + r] = m[r][NC - 1];
        }
    }
    __syncthreads();
    // a singular well block or a missing diagonal block: the host reports it
    // and nothing is updated
    if (s_bad[0] != 0x7fffffff || s_bad[1] != 0x7fffffff) return;
    const int lane = threadIdx.x;
    const bool on = lane < n1 * n1;
    const int r = on ? lane / n1 : 0, c = on ? lane % n1 : 0;
    for (int w = 0; w < nwells; ++w) {
        const int cell = wcell[w];
        int e = rp[cell];
        while (ci[e] != cell) ++e;         // present: checked above
        if (on) {
            double v = A[((size_t)e * n1 + r) * n1 + c];
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                v -= J1w[((size_t)w * n1 + r) * NW + k] * Qw[((size_t)w * NW + k) * n1 + c];
                if (c == 0) t += J1w[((size_t)w * n1 + r) * NW + k] * qw[(size_t)w * NW + k];
            }
            A[((size_t)e * n1 + r) * n1 + c] = v;
            if (c == 0) b[(size_t)cell * n1 + r] += t;
        }
        __syncthreads();
    }
}

// dw_w[k] = -qw_w[k] - sum_c Qw_w[k][c] d1_{c_w}[c], one thread per well unknown
__global__ void k_recover_wells(int nwells, int n1, int nw, const int *__restrict__ wcell,
                                const double *__restrict__ Qw, const double *__restrict__ qw,
                                const double *__restrict__ d1, double *__restrict__ dw) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nwells * nw) return;
    const int w = (int)(t / nw), k = (int)(t % nw);
    const double *Qk = Qw + ((size_t)w * nw + k) * n1;
    const double *x = d1 + (size_t)wcell[w] * n1;
    double s = -qw[t];
    for (int c = 0; c < n1; ++c) s -= Qk[c] * x[c];
    dw[t] = s;
}

void launch_condense_wells(int nwells, int n1, int nw, const int *rp, const int *ci, const int *wcell,
                           const double *J1w, const double *Jw1, const double *Jww, const double *rw, double *A,
                           double *b, double *Qw, double *qw, int *flag, hipStream_t st) {
    if (nwells == 0) return;
#define CASE(NN) case NN: hipLaunchKernelGGL(k_condense_wells<NN>, dim3(1), dim3(WL_THREADS), 0, st, nwells, n1, rp, ci, wcell, J1w, Jw1, Jww, rw, A, b, Qw, qw, flag); break;
    switch (nw) { CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "nw must be 1..8"); }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

void launch_recover_wells(int nwells, int n1, int nw, const int *wcell, const double *Qw, const double *qw,
                          const double *d1, double *dw, hipStream_t st) {
    if (nwells == 0) return;
    hipLaunchKernelGGL(k_recover_wells, dim3((unsigned)(((long)nwells * nw + 255) / 256)), dim3(256), 0, st, nwells,
                       n1, nw, wcell, Qw, qw, d1, dw);
    CPTR_CHECK_LAUNCH();
}

void launch_condense_cells(int n, int n1, int n2, const double *J21, const double *J22, const double *r2, double *Q,
                           double *q, int *flag, hipStream_t st) {
    if (n == 0 || n2 == 0) return;
    const dim3 grid((unsigned)(((long)n * CD_G + 255) / 256));
#define CASE(NN) case NN: hipLaunchKernelGGL(k_condense_cells<NN>, grid, dim3(256), 0, st, n, n1, J21, J22, r2, Q, q, flag); break;
    switch (n2) { CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "n2 must be 0..8"); }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

void launch_condense_blocks(int n, int n1, int n2, const int *rp, const int *ci, const double *J11, const double *J12,
                            const double *Q, const double *q, const double *r1, double *A, double *b,
                            hipStream_t st) {
    if (n == 0) return;
#define CASE(NN) case NN: hipLaunchKernelGGL(k_condense_blocks<NN>, dim3(n), dim3(64), 0, st, n, n1, rp, ci, J11, J12, Q, q, r1, A, b); break;
    switch (n2) { CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "n2 must be 0..8"); }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

void launch_condense_recover(int n, int n1, int n2, const double *Q, const double *q, const double *d1, double *d2,
                             hipStream_t st) {
    if (n == 0 || n2 == 0) return;
    hipLaunchKernelGGL(k_condense_recover, dim3((unsigned)(((long)n * n2 + 255) / 256)), dim3(256), 0, st, n, n1, n2,
                       Q, q, d1, d2);
    CPTR_CHECK_LAUNCH();
}

}  // namespace cptr
