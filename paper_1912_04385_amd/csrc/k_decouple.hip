// Left decoupling N^{-1} (Eq. splitPrec1) of the CPTR3 scheme (Eqs. CPTR31,
// CPTR32) and of CPR (Eq. CPR), and extraction of the scalar subsystems
// B_PP, C_TT and of the P / T column slabs used by Algorithm 2's residual
// updates.  Built with floating-point contraction off: the scaled matrix, and
// through it the AMG hierarchies, are reproducible bit for bit from the
// definition's evaluation order (stated at each formula).
#include "internal.h"

#include <algorithm>

namespace cptr {

// index of the k-th unknown of the eliminated group: the unknowns other than
// P (and T unless the group contains it), in ascending order
__device__ inline int group_index(int k, int ip, int it, bool with_t) {
    int lo = with_t ? ip : min(ip, it), hi = with_t ? -1 : max(ip, it);
    int g = k;
    if (g >= lo) ++g;
    if (hi >= 0 && g >= hi) ++g;
    return g;
}

// Phase 1, one thread per cell: solve the small system
// D_gg^T [w_P w_T] = [D_Pg^T D_Tg^T] (g = the eliminated group: s for CPTR3,
// s u {T} for CPR) by Gaussian elimination with partial pivoting -- first
// largest |pivot|, kij order, back substitution in descending rows -- and
//   CPTR3: beta = Ahat_ii[T][P] / Ahat_ii[P][P] (the two-stage CPTR scheme
//   keeps the first scaling alone: beta = 0, Abar[T] = Ahat[T]),
// with Ahat[P][c] = A[P][c] - sum_{k ascending} w_P[k] A[g_k][c] and
// Ahat[T][c] likewise with w_T.  w_P, w_T are stored by unknown (0 outside
// the group).  The same thread extracts B_PP = Abar[P,P] and
// C_TT = Abar[T,T] (Abar[T][c] = Ahat[T][c] - beta Ahat[P][c] for CPTR3), the
// only parts of the scaled matrix that the AMG setups need, so that they can
// start while phase 2 scales the whole matrix.
template <int B, int VAR>
struct DW {
    static constexpr bool CPR = (VAR == CPTR_VARIANT_CPR);
    static constexpr int NG = CPR ? B - 1 : B - 2;     // the eliminated group's size
    static constexpr int NR = CPR ? 1 : 2;             // right-hand sides: w_P (and w_T)
    static constexpr int NGX = NG > 0 ? NG : 1;
};

// The cell's solve from its diagonal block D (row-major B x B, any address
// space): F[k][0] = w_P[g_k], F[k][NR - 1] = w_T[g_k], and beta (CPTR3).
// False when a pivot is zero or Ahat_ii[P][P] is.
template <int B, int VAR>
__device__ inline bool dw_cell_solve(const double *D, int ip, int it, double (&F)[DW<B, VAR>::NGX][DW<B, VAR>::NR],
                                     double &bt) {
    constexpr bool CPR = DW<B, VAR>::CPR;
    constexpr int NG = DW<B, VAR>::NG, NR = DW<B, VAR>::NR, NGX = DW<B, VAR>::NGX;
    double M[NGX][NGX];
#pragma unroll
    for (int r = 0; r < NG; ++r) {
        const int gr = group_index(r, ip, it, CPR);
#pragma unroll
        for (int c = 0; c < NG; ++c) M[r][c] = D[group_index(c, ip, it, CPR) * B + gr];
        F[r][0] = D[ip * B + gr];
        if (NR == 2) F[r][NR - 1] = D[it * B + gr];
    }
    bool singular = false;
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        int p = k;
        double best = fabs(M[k][k]);
#pragma unroll
        for (int r = k + 1; r < NG; ++r) {
            const double a = fabs(M[r][k]);
            if (a > best) { best = a; p = r; }
        }
        if (best == 0.0) singular = true;
#pragma unroll
        for (int r = k + 1; r < NG; ++r) {
            if (r == p) {
#pragma unroll
                for (int c = 0; c < NG; ++c) { double t = M[k][c]; M[k][c] = M[r][c]; M[r][c] = t; }
#pragma unroll
                for (int j = 0; j < NR; ++j) { double t = F[k][j]; F[k][j] = F[r][j]; F[r][j] = t; }
            }
        }
#pragma unroll
        for (int r = k + 1; r < NG; ++r) {
            const double l = M[r][k] / M[k][k];
#pragma unroll
            for (int c = k + 1; c < NG; ++c) M[r][c] = M[r][c] - l * M[k][c];
#pragma unroll
            for (int j = 0; j < NR; ++j) F[r][j] = F[r][j] - l * F[k][j];
        }
    }
    if (singular) return false;
#pragma unroll
    for (int k = NG - 1; k >= 0; --k) {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
            double t = F[k][j];
#pragma unroll
            for (int c = k + 1; c < NG; ++c) t = t - M[k][c] * F[c][j];
            F[k][j] = t / M[k][k];
        }
    }
    bt = 0.0;
    if (VAR == CPTR_VARIANT_CPTR3) {
        double hp = D[ip * B + ip], ht = D[it * B + ip];
#pragma unroll
        for (int k = 0; k < NG; ++k) hp = hp - F[k][0] * D[group_index(k, ip, it, CPR) * B + ip];
#pragma unroll
        for (int k = 0; k < NG; ++k) ht = ht - F[k][NR - 1] * D[group_index(k, ip, it, CPR) * B + ip];
        if (hp == 0.0) return false;
        bt = ht / hp;
    }
    return true;
}

// w_P, w_T stored by unknown (0 outside the group) and beta
template <int B, int VAR>
__device__ inline void dw_store_weights(int i, int ip, int it, const double (&F)[DW<B, VAR>::NGX][DW<B, VAR>::NR],
                                        double bt, double *__restrict__ wp, double *__restrict__ wt,
                                        double *__restrict__ beta) {
    constexpr bool CPR = DW<B, VAR>::CPR;
    constexpr int NG = DW<B, VAR>::NG, NR = DW<B, VAR>::NR;
#pragma unroll
    for (int u = 0; u < B; ++u) {
        double vp = 0.0, vt = 0.0;
#pragma unroll
        for (int k = 0; k < NG; ++k)
            if (group_index(k, ip, it, CPR) == u) { vp = F[k][0]; vt = (NR == 2) ? F[k][NR - 1] : 0.0; }
        wp[(size_t)i * B + u] = vp;
        wt[(size_t)i * B + u] = vt;
    }
    beta[i] = bt;
}

// B_PP and C_TT entries of one block of the cell's row from the block's P
// and T columns: cP[r * stride] = A_ij[r][P], cT[r * stride] = A_ij[r][T]
template <int B, int VAR>
__device__ inline void dw_block_entries(const double *cP, const double *cT, int stride, int ip, int it,
                                        const double (&F)[DW<B, VAR>::NGX][DW<B, VAR>::NR], double bt,
                                        double &out_bpp, double &out_ctt) {
    constexpr bool CPR = DW<B, VAR>::CPR;
    constexpr int NG = DW<B, VAR>::NG, NR = DW<B, VAR>::NR;
    // Abar[P][P]: the P row at column P
    double hpP = cP[ip * stride];
#pragma unroll
    for (int k = 0; k < NG; ++k) hpP = hpP - F[k][0] * cP[group_index(k, ip, it, CPR) * stride];
    out_bpp = hpP;
    if (CPR) {
        out_ctt = cT[it * stride];       // T is in the eliminated group: its row is unchanged
    } else {
        double hpT = cT[ip * stride], htT = cT[it * stride];
#pragma unroll
        for (int k = 0; k < NG; ++k) hpT = hpT - F[k][0] * cT[group_index(k, ip, it, CPR) * stride];
#pragma unroll
        for (int k = 0; k < NG; ++k) htT = htT - F[k][NR - 1] * cT[group_index(k, ip, it, CPR) * stride];
        out_ctt = (VAR == CPTR_VARIANT_CPTR3) ? htT - bt * hpT : htT;
    }
}

template <int B, int VAR>
__global__ void __launch_bounds__(128) k_decouple_weights(int n, const int *__restrict__ rp,
                                                          const int *__restrict__ ci, const double *__restrict__ A,
                                                          int ip, int it, double *__restrict__ wp,
                                                          double *__restrict__ wt, double *__restrict__ beta, int *err,
                                                          double *__restrict__ ctt, double *__restrict__ bpp,
                                                          int *__restrict__ ee_rp, int *__restrict__ ee_ci,
                                                          double *__restrict__ ee_v) {
    constexpr bool CPR = DW<B, VAR>::CPR;
    constexpr int NG = DW<B, VAR>::NG, NR = DW<B, VAR>::NR, NGX = DW<B, VAR>::NGX;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int d = -1;
    for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (ci[e] == i) d = e;
    if (d < 0) {
        atomicMin(err, i);
        return;
    }
    double F[NGX][NR];
    double bt;
    if (!dw_cell_solve<B, VAR>(A + (size_t)d * B * B, ip, it, F, bt)) {
        atomicMin(err, i);
        return;
    }
    dw_store_weights<B, VAR>(i, ip, it, F, bt, wp, wt, beta);
    if (VAR == CPTR_VARIANT_CPTR && ee_v) {
        // the elliptic block B_ee straight from the weights (row u n + i at
        // 2 (u nnzb + rp[i]): P-block columns, then T-block columns + n),
        // each entry evaluated in the order of the apply phase
        const int nnzb = rp[n], e0 = rp[i], cnt = rp[i + 1] - e0;
        const size_t bp = 2 * (size_t)e0, bt2 = 2 * ((size_t)nnzb + e0);
        ee_rp[i] = (int)bp;
        ee_rp[n + i] = (int)bt2;
        if (i == n - 1) ee_rp[2 * n] = 4 * nnzb;
        for (int t = 0; t < cnt; ++t) {
            const int e = e0 + t;
            const double *Bk = A + (size_t)e * B * B;
            double pP = Bk[ip * B + ip], pT = Bk[ip * B + it], tP = Bk[it * B + ip], tT = Bk[it * B + it];
#pragma unroll
            for (int k = 0; k < NG; ++k) {
                const int g = group_index(k, ip, it, CPR);
                pP = pP - F[k][0] * Bk[g * B + ip];
                pT = pT - F[k][0] * Bk[g * B + it];
                tP = tP - F[k][NR - 1] * Bk[g * B + ip];
                tT = tT - F[k][NR - 1] * Bk[g * B + it];
            }
            const int c = ci[e];
            ee_ci[bp + t] = c;
            ee_v[bp + t] = pP;
            ee_ci[bp + cnt + t] = c + n;
            ee_v[bp + cnt + t] = pT;
            ee_ci[bt2 + t] = c;
            ee_v[bt2 + t] = tP;
            ee_ci[bt2 + cnt + t] = c + n;
            ee_v[bt2 + cnt + t] = tT;
        }
    }
    if (!ctt && !bpp) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const double *Bk = A + (size_t)e * B * B;
        double vb, vc;
        dw_block_entries<B, VAR>(Bk + ip, Bk + it, B, ip, it, F, bt, vb, vc);
        if (bpp) bpp[e] = vb;
        if (ctt) ctt[e] = vc;
    }
}

// Phase 1 for CPTR3 and CPR with the non-finite scan of the values folded
// in: one group of 8 lanes per cell, lane r reading row r of every block of
// the cell's row (so the block stream is read once, in contiguous rows, and
// every value is checked: flag bit 16).  The diagonal block and the P and T
// columns of up to DW_MAXB blocks go to LDS; one lane solves the cell as
// above, then one lane per block forms its B_PP and C_TT entries -- the same
// arithmetic as the one-thread-per-cell kernel, bit for bit.  Rows with more
// blocks take that kernel's path on the group's first lane.
constexpr int DW_CELLS = 32;     // cells per 256-thread workgroup
constexpr int DW_MAXB = 6;

template <int B, int VAR>
__global__ void __launch_bounds__(256) k_decouple_weights_rows(int n, const int *__restrict__ rp,
                                                               const int *__restrict__ ci,
                                                               const double *__restrict__ A, int ip, int it,
                                                               double *__restrict__ wp, double *__restrict__ wt,
                                                               double *__restrict__ beta, int *err, int *nf,
                                                               double *__restrict__ ctt, double *__restrict__ bpp) {
    constexpr int NG = DW<B, VAR>::NG, NR = DW<B, VAR>::NR, NGX = DW<B, VAR>::NGX;
    __shared__ double sD[DW_CELLS][B * B];
    __shared__ double sP[DW_CELLS][DW_MAXB][B];
    __shared__ double sT[DW_CELLS][DW_MAXB][B];
    __shared__ double sF[DW_CELLS][NGX][NR];
    __shared__ double sBt[DW_CELLS];
    __shared__ int sOk[DW_CELLS];
    const int g = threadIdx.x >> 3, r = threadIdx.x & 7;
    const int i = blockIdx.x * DW_CELLS + g;
    const bool act = i < n;
    int e0 = 0, nb = 0;
    if (act) {
        e0 = rp[i];
        nb = rp[i + 1] - e0;
    }
    // the diagonal block: the row's last entry in column i
    int dq = -1;
    for (int q = r; act && q < nb; q += 8)
        if (ci[e0 + q] == i) dq = q;
#pragma unroll
    for (int w = 4; w >= 1; w >>= 1) dq = max(dq, __shfl_xor(dq, w, 8));
    const bool staged = act && dq >= 0 && nb <= DW_MAXB;
    bool bad = false;
    if (act && r < B) {
        // the first DW_MAXB blocks with all their loads issued together
        double v[DW_MAXB][B];
#pragma unroll
        for (int q = 0; q < DW_MAXB; ++q) {
            const double *row = A + ((size_t)(e0 + q) * B + r) * B;
#pragma unroll
            for (int c = 0; c < B; ++c) v[q][c] = (q < nb) ? row[c] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < DW_MAXB; ++q) {
#pragma unroll
            for (int c = 0; c < B; ++c) bad = bad || !isfinite(v[q][c]);
            if (staged && q < nb) {
                if (q == dq) {
#pragma unroll
                    for (int c = 0; c < B; ++c) sD[g][r * B + c] = v[q][c];
                }
                const double *row = A + ((size_t)(e0 + q) * B + r) * B;
                sP[g][q][r] = row[ip];
                sT[g][q][r] = row[it];
            }
        }
        for (int q = DW_MAXB; q < nb; ++q) {
            const double *row = A + ((size_t)(e0 + q) * B + r) * B;
#pragma unroll
            for (int c = 0; c < B; ++c) bad = bad || !isfinite(row[c]);
        }
    }
    if (__ballot(bad) != 0 && (threadIdx.x & 63) == 0) atomicOr(nf, 16);
    __syncthreads();
    if (act && r == 0) {
        int ok = 0;
        if (dq < 0) {
            atomicMin(err, i);
        } else {
            const double *D = staged ? &sD[g][0] : A + (size_t)(e0 + dq) * B * B;
            double F[NGX][NR];
            double bt;
            if (!dw_cell_solve<B, VAR>(D, ip, it, F, bt)) {
                atomicMin(err, i);
            } else {
                dw_store_weights<B, VAR>(i, ip, it, F, bt, wp, wt, beta);
                if (staged) {
                    ok = 1;
#pragma unroll
                    for (int k = 0; k < NGX; ++k)
#pragma unroll
                        for (int j = 0; j < NR; ++j) sF[g][k][j] = F[k][j];
                    sBt[g] = bt;
                } else {
                    for (int e = e0; e < e0 + nb; ++e) {
                        const double *Bk = A + (size_t)e * B * B;
                        double vb, vc;
                        dw_block_entries<B, VAR>(Bk + ip, Bk + it, B, ip, it, F, bt, vb, vc);
                        bpp[e] = vb;
                        ctt[e] = vc;
                    }
                }
            }
        }
        sOk[g] = ok;
    }
    __syncthreads();
    if (act && r < nb && sOk[g]) {
        double F[NGX][NR];
#pragma unroll
        for (int k = 0; k < NGX; ++k)
#pragma unroll
            for (int j = 0; j < NR; ++j) F[k][j] = sF[g][k][j];
        double vb, vc;
        dw_block_entries<B, VAR>(&sP[g][r][0], &sT[g][r][0], 1, ip, it, F, sBt[g], vb, vc);
        bpp[e0 + r] = vb;
        ctt[e0 + r] = vc;
    }
}

// In-tile neighbour slot of cell i's block in column j (0 S, 1 W, 2 E, 3 N;
// -1 when j is not one of them or lies in another tx x ty tile)
__device__ inline int tile_slot(int i, int j, int nx, int tx, int ty) {
    const int x = i % nx, y = i / nx, xj = j % nx, yj = j / nx;
    if (xj / tx != x / tx || yj / ty != y / ty) return -1;
    if (yj == y - 1 && xj == x) return 0;
    if (yj == y && xj == x - 1) return 1;
    if (yj == y && xj == x + 1) return 2;
    if (yj == y + 1 && xj == x) return 3;
    return -1;
}

// Phase 2, one wavefront per cell, lane = block entry (r, c) = (lane / b,
// lane % b) of every block of the row, with the stored weights:
//   Abar[P][c] = Ahat[P][c],  Abar[T][c] = Ahat[T][c] - beta Ahat[P][c] (CPTR3),
// other rows copied; also the T and P column slabs and the FP32 copies.
template <int B, int VAR>
__global__ void __launch_bounds__(64) k_decouple_apply(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                       const double *__restrict__ A, int ip, int it,
                                                       const double *__restrict__ wp, const double *__restrict__ wt,
                                                       const double *__restrict__ beta, double *__restrict__ abar,
                                                       double *__restrict__ slabT, double *__restrict__ slabP,
                                                       float *__restrict__ abar32, float *__restrict__ slabT32,
                                                       float *__restrict__ slabP32, int nx, int tx, int ty,
                                                       float *__restrict__ tb32, double *__restrict__ tb64) {
    constexpr bool CPR = (VAR == CPTR_VARIANT_CPR);
    constexpr int NG = CPR ? B - 1 : B - 2;
    constexpr int NR = CPR ? 1 : 2;
    constexpr int NGX = NG > 0 ? NG : 1;
    const int lane = threadIdx.x;
    if (lane >= B * B) return;
    const bool tiles = tb32 || tb64;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
    unsigned slots = 0;         // in-tile neighbour slots written for this cell
    double F[NGX][NR];
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        const int g = group_index(k, ip, it, CPR);
        F[k][0] = wp[(size_t)i * B + g];
        if (NR == 2) F[k][NR - 1] = wt[(size_t)i * B + g];
    }
    const double bt = beta[i];
    const int r = lane / B, c = lane % B;
    const bool rowP = (r == ip), rowT = (!CPR && r == it);
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const double *Bk = A + (size_t)e * B * B;
        double out;
        if (rowP || rowT) {
            double hp = Bk[ip * B + c];
#pragma unroll
            for (int k = 0; k < NG; ++k) hp = hp - F[k][0] * Bk[group_index(k, ip, it, CPR) * B + c];
            if (rowP) {
                out = hp;
            } else {
                double ht = Bk[it * B + c];
#pragma unroll
                for (int k = 0; k < NG; ++k) ht = ht - F[k][NR - 1] * Bk[group_index(k, ip, it, CPR) * B + c];
                out = (VAR == CPTR_VARIANT_CPTR3) ? ht - bt * hp : ht;
            }
        } else {
            out = Bk[r * B + c];
        }
        abar[(size_t)e * B * B + lane] = out;
        if (abar32) abar32[(size_t)e * B * B + lane] = (float)out;
        if (c == it) {
            if (slabT) slabT[(size_t)e * B + r] = out;
            if (slabT32) slabT32[(size_t)e * B + r] = (float)out;
        }
        if (c == ip) {
            if (slabP) slabP[(size_t)e * B + r] = out;
            if (slabP32) slabP32[(size_t)e * B + r] = (float)out;
        }
        if (tiles) {
            // the BILU(0) sweeps' side array: the block of an in-tile
            // neighbour (the row's first entry in that column)
            const int k = tile_slot(i, ci[e], nx, tx, ty);
            if (k >= 0 && !((slots >> k) & 1u)) {
                slots |= 1u << k;
                const size_t o = ((size_t)i * 4 + k) * B * B + lane;
                if (tb32) tb32[o] = (float)out;
                if (tb64) tb64[o] = out;
            }
        }
    }
    if (tiles) {
        for (int k = 0; k < 4; ++k) {
            if ((slots >> k) & 1u) continue;
            const size_t o = ((size_t)i * 4 + k) * B * B + lane;
            if (tb32) tb32[o] = 0.0f;
            if (tb64) tb64[o] = 0.0;
        }
    }
    }
}

void launch_decouple_weights(int variant, int n, int b, const int *rp, const int *ci, const double *A, int ip,
                             int it, double *wp, double *wt, double *beta, int *err, double *ctt, double *bpp,
                             int *ee_rp, int *ee_ci, double *ee_v, hipStream_t s) {
    if (ee_v && variant != CPTR_VARIANT_CPTR) throw Error(CPTR_E_ARG, "the elliptic block belongs to the two-stage variant");
    if (n == 0) return;
    const dim3 g((n + 127) / 128), t(128);
#define CASE(BB)                                                                                                  \
    case BB:                                                                                                      \
        if (variant == CPTR_VARIANT_CPR)                                                                          \
            hipLaunchKernelGGL((k_decouple_weights<BB, CPTR_VARIANT_CPR>), g, t, 0, s, n, rp, ci, A, ip, it, wp,  \
                               wt, beta, err, ctt, bpp, ee_rp, ee_ci, ee_v);                                      \
        else if (variant == CPTR_VARIANT_CPTR)                                                                    \
            hipLaunchKernelGGL((k_decouple_weights<BB, CPTR_VARIANT_CPTR>), g, t, 0, s, n, rp, ci, A, ip, it, wp,  \
                               wt, beta, err, ctt, bpp, ee_rp, ee_ci, ee_v);                                      \
        else                                                                                                      \
            hipLaunchKernelGGL((k_decouple_weights<BB, CPTR_VARIANT_CPTR3>), g, t, 0, s, n, rp, ci, A, ip, it, wp, \
                               wt, beta, err, ctt, bpp, ee_rp, ee_ci, ee_v);                                      \
        break;
    switch (b) {
        CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        default: throw Error(CPTR_E_ARG, "block size must be 2..8");
    }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

void launch_decouple_weights_rows(int variant, int n, int b, const int *rp, const int *ci, const double *A, int ip,
                                  int it, double *wp, double *wt, double *beta, int *err, int *nf, double *ctt,
                                  double *bpp, hipStream_t s) {
    if (variant != CPTR_VARIANT_CPTR3 && variant != CPTR_VARIANT_CPR)
        throw Error(CPTR_E_ARG, "the row kernel of the decoupling takes CPTR3 and CPR only");
    if (n == 0) return;
    const dim3 g((unsigned)((n + DW_CELLS - 1) / DW_CELLS)), t(256);
#define CASE(BB)                                                                                                  \
    case BB:                                                                                                      \
        if (variant == CPTR_VARIANT_CPR)                                                                          \
            hipLaunchKernelGGL((k_decouple_weights_rows<BB, CPTR_VARIANT_CPR>), g, t, 0, s, n, rp, ci, A, ip, it, \
                               wp, wt, beta, err, nf, ctt, bpp);                                                  \
        else                                                                                                      \
            hipLaunchKernelGGL((k_decouple_weights_rows<BB, CPTR_VARIANT_CPTR3>), g, t, 0, s, n, rp, ci, A, ip,   \
                               it, wp, wt, beta, err, nf, ctt, bpp);                                              \
        break;
    switch (b) {
        CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        default: throw Error(CPTR_E_ARG, "block size must be 2..8");
    }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

// The apply phase runs beside the AMG setups: its grid is capped so that it
// holds a quarter of the GPU's wavefront slots and leaves room for their
// kernels (each wavefront loops over cells).
constexpr int DA_MAX_WAVES = 2048;

void launch_decouple_apply(int variant, int n, int b, const int *rp, const int *ci, const double *A, int ip, int it,
                           const double *wp, const double *wt, const double *beta, double *abar, double *slabT,
                           double *slabP, float *abar32, float *slabT32, float *slabP32, hipStream_t s, int nx,
                           int tx, int ty, float *tb32, double *tb64) {
    if (n == 0) return;
    const int grid = std::min(n, DA_MAX_WAVES);
#define CASE(BB)                                                                                                  \
    case BB:                                                                                                      \
        if (variant == CPTR_VARIANT_CPR)                                                                          \
            hipLaunchKernelGGL((k_decouple_apply<BB, CPTR_VARIANT_CPR>), dim3(grid), dim3(64), 0, s, n, rp, ci, A, \
                               ip, it, wp, wt, beta, abar, slabT, slabP, abar32, slabT32, slabP32, nx, tx, ty, tb32, tb64);              \
        else if (variant == CPTR_VARIANT_CPTR)                                                                    \
            hipLaunchKernelGGL((k_decouple_apply<BB, CPTR_VARIANT_CPTR>), dim3(grid), dim3(64), 0, s, n, rp, ci,   \
                               A, ip, it, wp, wt, beta, abar, slabT, slabP, abar32, slabT32, slabP32, nx, tx, ty, tb32, tb64);           \
        else                                                                                                      \
            hipLaunchKernelGGL((k_decouple_apply<BB, CPTR_VARIANT_CPTR3>), dim3(grid), dim3(64), 0, s, n, rp, ci,  \
                               A, ip, it, wp, wt, beta, abar, slabT, slabP, abar32, slabT32, slabP32, nx, tx, ty, tb32, tb64);           \
        break;
    switch (b) {
        CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
        default: throw Error(CPTR_E_ARG, "block size must be 2..8");
    }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

void launch_decouple(int variant, int n, int b, const int *rp, const int *ci, const double *A, int ip, int it,
                     double *abar, double *wp, double *wt, double *beta, int *err, hipStream_t s) {
    launch_decouple_weights(variant, n, b, rp, ci, A, ip, it, wp, wt, beta, err, nullptr, nullptr, nullptr, nullptr,
                            nullptr, s);
    launch_decouple_apply(variant, n, b, rp, ci, A, ip, it, wp, wt, beta, abar, nullptr, nullptr, nullptr, nullptr,
                          nullptr, s);
}

// bbar = N^{-1} b for one right-hand side, same order as the rows:
//   hp = b[P] - sum_{g ascending} w_P[g] b[g];  ht likewise;  T: ht - beta hp
// The stored w vectors are zero outside the group, and the sum skips the
// P and T positions (and T for CPR's P row) exactly like the group loop.
template <int B>
__global__ void k_scale_rhs(int variant, int n, const double *__restrict__ rhs, int ip, int it,
                            const double *__restrict__ wp, const double *__restrict__ wt,
                            const double *__restrict__ beta, double *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *bi = rhs + (size_t)i * B;
    double v[B];
    for (int r = 0; r < B; ++r) v[r] = bi[r];
    double hp = v[ip];
    for (int g = 0; g < B; ++g) {
        if (g == ip || (g == it && variant != CPTR_VARIANT_CPR)) continue;
        hp = hp - wp[(size_t)i * B + g] * v[g];
    }
    double o[B];
    for (int r = 0; r < B; ++r) o[r] = v[r];
    o[ip] = hp;
    if (variant != CPTR_VARIANT_CPR) {
        double ht = v[it];
        for (int g = 0; g < B; ++g) {
            if (g == ip || g == it) continue;
            ht = ht - wt[(size_t)i * B + g] * v[g];
        }
        o[it] = (variant == CPTR_VARIANT_CPTR3) ? ht - beta[i] * hp : ht;
    }
    for (int r = 0; r < B; ++r) out[(size_t)i * B + r] = o[r];
}

// v = N r: undo the scaling (second scaling first, then the first)
template <int B>
__global__ void k_unscale(int variant, int n, const double *__restrict__ rv, int ip, int it,
                          const double *__restrict__ wp, const double *__restrict__ wt,
                          const double *__restrict__ beta, double *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v[B];
    for (int r = 0; r < B; ++r) v[r] = rv[(size_t)i * B + r];
    if (variant == CPTR_VARIANT_CPTR3) v[it] = v[it] + beta[i] * v[ip];
    double sp = 0.0, st = 0.0;
    for (int g = 0; g < B; ++g) {
        if (g == ip || (g == it && variant != CPTR_VARIANT_CPR)) continue;
        sp += wp[(size_t)i * B + g] * v[g];
        if (variant != CPTR_VARIANT_CPR && g != it) st += wt[(size_t)i * B + g] * v[g];
    }
    double o[B];
    for (int r = 0; r < B; ++r) o[r] = v[r];
    o[ip] = v[ip] + sp;
    if (variant != CPTR_VARIANT_CPR) o[it] = v[it] + st;
    for (int r = 0; r < B; ++r) out[(size_t)i * B + r] = o[r];
}

void launch_scale_rhs(int variant, int n, int b, const double *rhs, int ip, int it, const double *wp,
                      const double *wt, const double *beta, double *out, hipStream_t s) {
    if (n == 0) return;
    dim3 g((n + 127) / 128), t(128);
#define CASE(BB) case BB: hipLaunchKernelGGL(k_scale_rhs<BB>, g, t, 0, s, variant, n, rhs, ip, it, wp, wt, beta, out); break;
    switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

void launch_unscale(int variant, int n, int b, const double *v, int ip, int it, const double *wp,
                    const double *wt, const double *beta, double *out, hipStream_t s) {
    if (n == 0) return;
    dim3 g((n + 127) / 128), t(128);
#define CASE(BB) case BB: hipLaunchKernelGGL(k_unscale<BB>, g, t, 0, s, variant, n, v, ip, it, wp, wt, beta, out); break;
    switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

// Scalar subsystems on the BSR pattern: C_TT = Abar[T,T] (Eq. CPTR32),
// B_PP = Abar[P,P] (Eq. CPTR31); column slabs slab_T[e*b + r] = Abar_e[r][T],
// slab_P[e*b + r] = Abar_e[r][P]; optional FP32 copies.
__global__ void k_extract(int nnzb, int b, const double *__restrict__ abar, int ip, int it, double *ctt,
                          double *bpp, double *slabT, double *slabP, float *abar32, float *slabT32,
                          float *slabP32) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)nnzb) return;
    const double *Bk = abar + e * b * b;
    if (ctt) ctt[e] = Bk[it * b + it];
    if (bpp) bpp[e] = Bk[ip * b + ip];
    for (int r = 0; r < b; ++r) {
        double vt = Bk[r * b + it], vp = Bk[r * b + ip];
        if (slabT) slabT[e * b + r] = vt;
        if (slabP) slabP[e * b + r] = vp;
        if (slabT32) slabT32[e * b + r] = (float)vt;
        if (slabP32) slabP32[e * b + r] = (float)vp;
    }
    if (abar32)
        for (int k = 0; k < b * b; ++k) abar32[e * b * b + k] = (float)Bk[k];
}

void launch_extract(int n, int b, int nnzb, const double *abar, int ip, int it, double *ctt, double *bpp,
                    double *slabT, double *slabP, float *abar32, float *slabT32, float *slabP32, hipStream_t s) {
    (void)n;
    if (nnzb == 0) return;
    hipLaunchKernelGGL(k_extract, dim3((nnzb + 255) / 256), dim3(256), 0, s, nnzb, b, abar, ip, it, ctt, bpp, slabT,
                       slabP, abar32, slabT32, slabP32);
    CPTR_CHECK_LAUNCH();
}

}  // namespace cptr
