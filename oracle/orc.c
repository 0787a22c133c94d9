/*
 * CPU FP64 oracle for the multi-stage (CPTR3 / CPTR / CPR) preconditioned
 * GMRES path.  TEST INFRASTRUCTURE ONLY: the product library never links,
 * loads or calls this file; tests, the smoke check and the CPU baseline leg
 * of the benchmark do.
 *
 * Plain, serial, slow on purpose.  Every routine states the passage of
 * Cremon, Castelletto & White (multi-stage preconditioners for
 * thermal-compositional-reactive flow) or the published algorithm it writes
 * out.  Floating point is IEEE double, built with -ffp-contract=off; where a
 * later integer decision depends on a value (AMG strength, coarsening,
 * truncation) the evaluation order is spelled out in the comment so that any
 * independent implementation of the same definition reaches the same bits.
 *
 * Conventions: BSR with int32 row pointers / ascending block columns and
 * row-major b x b blocks; CSR likewise.  Cell unknowns are indexed 0..b-1; the
 * pressure index ip and temperature index it are arguments, every other index
 * belongs to the "s" group (saturations / mole fractions) in ascending order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* dense Gaussian elimination with partial pivoting                          */
/* ------------------------------------------------------------------------ */

/* Solve M X = F in place (M: m x m row-major, F: m x nrhs row-major, X written
 * into F).  Textbook kij elimination: at step k the pivot is the first row
 * r >= k with the largest |M[r][k]|; rows k and p are swapped in M and F;
 * for r > k: l = M[r][k] / M[k][k], M[r][c] = M[r][c] - l*M[k][c] (c > k),
 * F[r][j] = F[r][j] - l*F[k][j].  Back substitution:
 * X[k][j] = (F[k][j] - sum_{c>k, ascending} M[k][c]*X[c][j]) / M[k][k].
 * Returns 0, or -1 when a pivot is exactly zero. */
static int gepp_solve(int m, double *M, int nrhs, double *F)
{
    for (int k = 0; k < m; ++k) {
        int p = k;
        double best = fabs(M[k * m + k]);
        for (int r = k + 1; r < m; ++r) {
            double a = fabs(M[r * m + k]);
            if (a > best) { best = a; p = r; }
        }
        if (best == 0.0) return -1;
        if (p != k) {
            for (int c = 0; c < m; ++c) { double t = M[k*m+c]; M[k*m+c] = M[p*m+c]; M[p*m+c] = t; }
            for (int j = 0; j < nrhs; ++j) { double t = F[k*nrhs+j]; F[k*nrhs+j] = F[p*nrhs+j]; F[p*nrhs+j] = t; }
        }
        for (int r = k + 1; r < m; ++r) {
            double l = M[r * m + k] / M[k * m + k];
            for (int c = k + 1; c < m; ++c) M[r * m + c] = M[r * m + c] - l * M[k * m + c];
            for (int j = 0; j < nrhs; ++j) F[r * nrhs + j] = F[r * nrhs + j] - l * F[k * nrhs + j];
        }
    }
    for (int k = m - 1; k >= 0; --k) {
        for (int j = 0; j < nrhs; ++j) {
            double t = F[k * nrhs + j];
            for (int c = k + 1; c < m; ++c) t = t - M[k * m + c] * F[c * nrhs + j];
            F[k * nrhs + j] = t / M[k * m + k];
        }
    }
    return 0;
}

/* Explicit inverse of a b x b block via gepp_solve with the identity as RHS. */
static int block_inverse(int b, const double *A, double *Ainv, double *work)
{
    memcpy(work, A, sizeof(double) * b * b);
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) Ainv[r * b + c] = (r == c) ? 1.0 : 0.0;
    return gepp_solve(b, work, b, Ainv);
}

/* C = A * B for b x b blocks, C[r][c] = sum_{k ascending} A[r][k]*B[k][c]. */
static void block_mul(int b, const double *A, const double *B, double *C)
{
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) {
            double t = 0.0;
            for (int k = 0; k < b; ++k) t = t + A[r * b + k] * B[k * b + c];
            C[r * b + c] = t;
        }
}

/* Dense LU with partial pivoting of the coarsest AMG level (a direct coarse
 * solve, as the paper's AMG uses): PA = LU stored in place, piv[k] = row
 * swapped with k at step k.  Same pivot rule as gepp_solve.  Returns 0 or -1. */
int orc_dense_lu_factor(int m, double *M, int *piv)
{
    for (int k = 0; k < m; ++k) {
        int p = k;
        double best = fabs(M[(size_t)k * m + k]);
        for (int r = k + 1; r < m; ++r) {
            double a = fabs(M[(size_t)r * m + k]);
            if (a > best) { best = a; p = r; }
        }
        piv[k] = p;
        if (best == 0.0) return -1;
        if (p != k)
            for (int c = 0; c < m; ++c) { double t = M[(size_t)k*m+c]; M[(size_t)k*m+c] = M[(size_t)p*m+c]; M[(size_t)p*m+c] = t; }
        for (int r = k + 1; r < m; ++r) {
            double l = M[(size_t)r * m + k] / M[(size_t)k * m + k];
            M[(size_t)r * m + k] = l;
            for (int c = k + 1; c < m; ++c) M[(size_t)r * m + c] = M[(size_t)r * m + c] - l * M[(size_t)k * m + c];
        }
    }
    return 0;
}

/* x = A^{-1} f with the factors of orc_dense_lu_factor (f overwritten) */
void orc_dense_lu_solve(int m, const double *M, const int *piv, double *f)
{
    for (int k = 0; k < m; ++k)
        if (piv[k] != k) { double t = f[k]; f[k] = f[piv[k]]; f[piv[k]] = t; }
    for (int r = 0; r < m; ++r) {
        double t = f[r];
        for (int c = 0; c < r; ++c) t = t - M[(size_t)r * m + c] * f[c];
        f[r] = t;
    }
    for (int r = m - 1; r >= 0; --r) {
        double t = f[r];
        for (int c = r + 1; c < m; ++c) t = t - M[(size_t)r * m + c] * f[c];
        f[r] = t / M[(size_t)r * m + r];
    }
}

/* ------------------------------------------------------------------------ */
/* left decoupling N^{-1}  (split preconditioning, Eq. splitPrec1)           */
/* ------------------------------------------------------------------------ */

static int find_diag(const int *rp, const int *ci, int i)
{
    for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (ci[e] == i) return e;
    return -1;
}

/*
 * Per-cell quasi-IMPES decoupling.  D = diag(.) extracts the cell-local
 * entries (remark on diagonal extraction), so N^{-1} is block diagonal with
 * one b x b factor per cell, applied to every block of the cell's block row
 * and to the cell's right-hand side.
 *
 * variant 0 (CPTR3, Eqs. CPTR31 and CPTR32):
 *   w_P^T = D_Ps D_ss^{-1},  w_T^T = D_Ts D_ss^{-1}   (solve D_ss^T w = D_.s^T)
 *   first scaling:  Ahat[P,:] = A[P,:] - sum_k w_P[k] A[s_k,:]
 *                   Ahat[T,:] = A[T,:] - sum_k w_T[k] A[s_k,:]
 *   second scaling: beta = Ahat_ii[T,P] / Ahat_ii[P,P]  (D_Tp D_PP^{-1} taken
 *                   from the once-scaled diagonal block)
 *                   Abar[T,:] = Ahat[T,:] - beta * Ahat[P,:]
 * variant 1 (CPR, Eq. CPR): h = s u {T};  w^T = D_Ph D_hh^{-1};
 *                   Abar[P,:] = A[P,:] - sum_{k in h ascending} w[k] A[h_k,:]
 * variant 2 (CPTR, Eq. CPTR1): the first CPTR3 scaling alone (e = {P, T}).
 * Rows of the s group are unchanged in every variant.
 *
 * Evaluation order (mirrored bit for bit by any faithful implementation):
 *   t = A[P][c]; for k ascending: t = t - w[k]*A[s_k][c];  likewise for T;
 *   Abar[T][c] = that - beta * Ahat[P][c].
 *
 * Outputs: Abar (nnzb*b*b), rhsbar (n*b), and per cell the factors
 * wp[n*b], wt[n*b] (coefficient of row r in the P / T combination, zero for
 * r not in the eliminated group) and beta[n].  Returns 0 or -(1+cell) when a
 * cell's D_ss (D_hh) is singular or Ahat_ii[P,P] is zero.
 */
int orc_decouple(int variant, int n, int b, const int *rp, const int *ci,
                 const double *A, const double *rhs, int ip, int it,
                 double *Abar, double *rhsbar, double *wp, double *wt, double *beta)
{
    int grp[64];           /* indices eliminated against */
    int ng = 0;
    for (int r = 0; r < b; ++r) {
        if (r == ip) continue;
        if (r == it && variant != 1) continue;
        grp[ng++] = r;
    }
    double M[64 * 64], F[64 * 2];
    for (int i = 0; i < n; ++i) {
        int d = find_diag(rp, ci, i);
        if (d < 0) return -(1 + i);
        const double *D = A + (size_t)d * b * b;
        int nrhs = (variant == 1) ? 1 : 2;
        for (int r = 0; r < ng; ++r) {
            for (int c = 0; c < ng; ++c) M[r * ng + c] = D[grp[c] * b + grp[r]];  /* D_gg^T */
            F[r * nrhs + 0] = D[ip * b + grp[r]];
            if (nrhs == 2) F[r * nrhs + 1] = D[it * b + grp[r]];
        }
        if (ng > 0 && gepp_solve(ng, M, nrhs, F) != 0) return -(1 + i);
        double *wpi = wp + (size_t)i * b, *wti = wt + (size_t)i * b;
        for (int r = 0; r < b; ++r) { wpi[r] = 0.0; wti[r] = 0.0; }
        for (int k = 0; k < ng; ++k) {
            wpi[grp[k]] = F[k * nrhs + 0];
            if (nrhs == 2) wti[grp[k]] = F[k * nrhs + 1];
        }
        /* once-scaled diagonal block entries needed for beta */
        double bt = 0.0;
        if (variant == 0) {
            double hp = D[ip * b + ip], ht = D[it * b + ip];
            for (int k = 0; k < ng; ++k) hp = hp - F[k * nrhs + 0] * D[grp[k] * b + ip];
            for (int k = 0; k < ng; ++k) ht = ht - F[k * nrhs + 1] * D[grp[k] * b + ip];
            if (hp == 0.0) return -(1 + i);
            bt = ht / hp;
        }
        beta[i] = bt;
        /* apply to every block of the row, then to the rhs (treated as one more column) */
        for (int e = rp[i]; e <= rp[i + 1]; ++e) {
            const double *B; double *O; int ncol, ld;
            if (e < rp[i + 1]) { B = A + (size_t)e * b * b; O = Abar + (size_t)e * b * b; ncol = b; ld = b; }
            else { B = rhs + (size_t)i * b; O = rhsbar + (size_t)i * b; ncol = 1; ld = 1; }
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < ncol; ++c) O[r * ld + c] = B[r * ld + c];
            for (int c = 0; c < ncol; ++c) {
                double hp = B[ip * ld + c];
                for (int k = 0; k < ng; ++k) hp = hp - F[k * nrhs + 0] * B[grp[k] * ld + c];
                O[ip * ld + c] = hp;
                if (variant != 1) {
                    double ht = B[it * ld + c];
                    for (int k = 0; k < ng; ++k) ht = ht - F[k * nrhs + 1] * B[grp[k] * ld + c];
                    if (variant == 0) ht = ht - bt * hp;
                    O[it * ld + c] = ht;
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* sparse products                                                           */
/* ------------------------------------------------------------------------ */

/* y = A x for BSR A; y_i[r] = sum_{blocks e ascending} sum_{c ascending} A_e[r][c] x_col[c] */
void orc_bsr_spmv(int n, int b, const int *rp, const int *ci, const double *A,
                  const double *x, double *y)
{
    for (int i = 0; i < n; ++i)
        for (int r = 0; r < b; ++r) {
            double t = 0.0;
            for (int e = rp[i]; e < rp[i + 1]; ++e) {
                const double *B = A + (size_t)e * b * b + r * b;
                const double *xc = x + (size_t)ci[e] * b;
                for (int c = 0; c < b; ++c) t = t + B[c] * xc[c];
            }
            y[(size_t)i * b + r] = t;
        }
}

/* y = A x for CSR A */
void orc_csr_spmv(int n, const int *rp, const int *ci, const double *v, const double *x, double *y)
{
    for (int i = 0; i < n; ++i) {
        double t = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) t = t + v[e] * x[ci[e]];
        y[i] = t;
    }
}

/* B = A^T (A: nr x nc CSR).  Rows of B list their columns ascending. */
void orc_csr_transpose(int nr, int nc, const int *rp, const int *ci, const double *v,
                       int *rpT, int *ciT, double *vT)
{
    for (int j = 0; j <= nc; ++j) rpT[j] = 0;
    for (int e = 0; e < rp[nr]; ++e) rpT[ci[e] + 1]++;
    for (int j = 0; j < nc; ++j) rpT[j + 1] += rpT[j];
    int *next = (int *)malloc(sizeof(int) * (nc > 0 ? nc : 1));
    for (int j = 0; j < nc; ++j) next[j] = rpT[j];
    for (int i = 0; i < nr; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int p = next[ci[e]]++;
            ciT[p] = i;
            vT[p] = v[e];
        }
    free(next);
}

/* Gustavson C = A B, symbolic part: number of distinct columns per row. */
int orc_spgemm_count(int m, int ncb, const int *arp, const int *aci,
                     const int *brp, const int *bci, int *crp)
{
    int *mark = (int *)malloc(sizeof(int) * (ncb > 0 ? ncb : 1));
    for (int j = 0; j < ncb; ++j) mark[j] = -1;
    crp[0] = 0;
    for (int i = 0; i < m; ++i) {
        int cnt = 0;
        for (int e = arp[i]; e < arp[i + 1]; ++e) {
            int k = aci[e];
            for (int f = brp[k]; f < brp[k + 1]; ++f) {
                int j = bci[f];
                if (mark[j] != i) { mark[j] = i; cnt++; }
            }
        }
        crp[i + 1] = crp[i] + cnt;
    }
    free(mark);
    return crp[m];
}

/* Gustavson numeric part.  For each output entry (i, j) the terms a_ik*b_kj
 * are added in ascending k (A's row order), starting from the first term:
 * c = a_ik1*b_k1j; c = c + a_ik2*b_k2j; ...  Output columns ascending.
 * Every (i, j) reached structurally is stored, even if its value is zero. */
void orc_spgemm_fill(int m, int ncb, const int *arp, const int *aci, const double *av,
                     const int *brp, const int *bci, const double *bv,
                     const int *crp, int *cci, double *cv)
{
    int *pos = (int *)malloc(sizeof(int) * (ncb > 0 ? ncb : 1));
    for (int j = 0; j < ncb; ++j) pos[j] = -1;
    for (int i = 0; i < m; ++i) {
        int base = crp[i], cnt = 0;
        for (int e = arp[i]; e < arp[i + 1]; ++e) {
            int k = aci[e];
            double a = av[e];
            for (int f = brp[k]; f < brp[k + 1]; ++f) {
                int j = bci[f];
                double t = a * bv[f];
                if (pos[j] < 0) { pos[j] = base + cnt; cci[base + cnt] = j; cv[base + cnt] = t; cnt++; }
                else cv[pos[j]] = cv[pos[j]] + t;
            }
        }
        /* insertion sort of the row by column */
        for (int p = base + 1; p < base + cnt; ++p) {
            int cj = cci[p]; double vj = cv[p]; int q = p - 1;
            while (q >= base && cci[q] > cj) { cci[q + 1] = cci[q]; cv[q + 1] = cv[q]; --q; }
            cci[q + 1] = cj; cv[q + 1] = vj;
        }
        for (int p = base; p < base + cnt; ++p) pos[cci[p]] = -1;
    }
    free(pos);
}

/* ------------------------------------------------------------------------ */
/* classical AMG setup pieces                                                */
/* ------------------------------------------------------------------------ */

/* Strength of connection (sign-aware classical criterion).  With
 * sigma_i = -1 if a_ii < 0 else +1 and m_i = max_{k != i} (-sigma_i a_ik):
 * j != i is a strong dependence of i iff m_i > 0 and -sigma_i a_ij >= theta*m_i.
 * s[e] is 1 for strong off-diagonal entries, else 0. */
void orc_strength(int n, const int *rp, const int *ci, const double *v, double theta,
                  unsigned char *s)
{
    for (int i = 0; i < n; ++i) {
        double aii = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) if (ci[e] == i) aii = v[e];
        double sg = (aii < 0.0) ? -1.0 : 1.0;
        double m = 0.0; int any = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            if (ci[e] == i) continue;
            double t = -sg * v[e];
            if (!any || t > m) { m = t; any = 1; }
        }
        double thr = theta * m;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            s[e] = 0;
            if (ci[e] == i || !any || !(m > 0.0)) continue;
            if (-sg * v[e] >= thr) s[e] = 1;
        }
    }
}

/* SplitMix64 (Steele, Lea & Flood, 2014): the output function applied to
 * the counter seed + (i+1) * golden gamma. */
uint64_t orc_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* does i win against j?  measure lambda = |S^T| + random in [0,1): compare
 * (|S^T|, random) lexicographically, then the lower index. */
static int beats(int i, int j, const int *cntT, const uint64_t *h)
{
    if (cntT[i] != cntT[j]) return cntT[i] > cntT[j];
    if (h[i] != h[j]) return h[i] > h[j];
    return i < j;
}

/* PMIS coarsening (De Sterck, Yang & Heys, 2006).
 *   lambda_i = |S^T_i| + rho_i (rho_i from SplitMix64); points with
 *   |S^T_i| = 0 (nobody depends on them) start as F.  Repeat: every undecided
 *   point that beats all undecided points of its symmetrised strong
 *   neighbourhood S_i u S^T_i becomes C (simultaneously); then every
 *   undecided point that strongly depends on one of the new C points becomes F.
 * cf[i] = 1 for C, 0 for F.  Returns the number of C points and the number of
 * rounds in *rounds. */
int orc_pmis(int n, const int *rp, const int *ci, const unsigned char *s, uint64_t seed,
             int *cf, int *rounds)
{
    int nnz = rp[n];
    int *cntT = (int *)calloc(n > 0 ? n : 1, sizeof(int));
    for (int e = 0; e < nnz; ++e) if (s[e]) cntT[ci[e]]++;
    /* S^T adjacency */
    int *tp = (int *)calloc(n + 1, sizeof(int));
    for (int e = 0; e < nnz; ++e) if (s[e]) tp[ci[e] + 1]++;
    for (int j = 0; j < n; ++j) tp[j + 1] += tp[j];
    int *tnext = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int *tadj = (int *)malloc(sizeof(int) * (tp[n] > 0 ? tp[n] : 1));
    for (int j = 0; j < n; ++j) tnext[j] = tp[j];
    for (int i = 0; i < n; ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) if (s[e]) tadj[tnext[ci[e]]++] = i;
    uint64_t *h = (uint64_t *)malloc(sizeof(uint64_t) * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) h[i] = orc_splitmix64(seed, (uint64_t)i);

    enum { UND = -1 };
    int *st = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    unsigned char *newc = (unsigned char *)calloc(n > 0 ? n : 1, 1);
    int und = 0;
    for (int i = 0; i < n; ++i) { st[i] = (cntT[i] == 0) ? 0 : UND; und += (st[i] == UND); }
    int nr = 0;
    while (und > 0) {
        nr++;
        for (int i = 0; i < n; ++i) {
            newc[i] = 0;
            if (st[i] != UND) continue;
            int win = 1;
            for (int e = rp[i]; e < rp[i + 1] && win; ++e)
                if (s[e] && st[ci[e]] == UND && !beats(i, ci[e], cntT, h)) win = 0;
            for (int f = tp[i]; f < tp[i + 1] && win; ++f)
                if (st[tadj[f]] == UND && !beats(i, tadj[f], cntT, h)) win = 0;
            newc[i] = (unsigned char)win;
        }
        for (int i = 0; i < n; ++i) if (newc[i]) { st[i] = 1; und--; }
        for (int i = 0; i < n; ++i) {
            if (st[i] != UND) continue;
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                if (s[e] && newc[ci[e]]) { st[i] = 0; und--; break; }
        }
    }
    int nc = 0;
    for (int i = 0; i < n; ++i) { cf[i] = st[i]; nc += st[i]; }
    if (rounds) *rounds = nr;
    free(cntT); free(tp); free(tnext); free(tadj); free(h); free(st); free(newc);
    return nc;
}

/* abar_kl of the extended+i formula: a_kl when it has the sign opposite to
 * a_kk, else 0 */
static double abar(double akk, double akl)
{
    if ((akk > 0.0 && akl < 0.0) || (akk < 0.0 && akl > 0.0)) return akl;
    return 0.0;
}

typedef struct {
    int *mark;      /* n, stamp: in C-hat of the current row */
    int *hat;       /* list of C-hat */
    double *w;      /* weights aligned with hat */
    int cap;
} exti_ws;

/*
 * Extended+i interpolation (De Sterck, Falgout, Nolting & Yang, 2008) for
 * one row.  For an F point i with strong C neighbours C_i^s and strong F
 * neighbours F_i^s, the interpolatory set is
 *   Chat_i = C_i^s  u  (strong C neighbours of every k in F_i^s)
 * and, with abar as above and d_k = sum_{l in Chat_i u {i}} abar_kl,
 *   w_ij = -( a_ij + sum_{k in F_i^s} a_ik abar_kj / d_k ) / atilde_ii,
 *   atilde_ii = a_ii + sum_{n weak, n not in Chat_i} a_in
 *                    + sum_{k in F_i^s} a_ik abar_ki / d_k.
 * Reading where the formula is silent: a k with d_k = 0 is lumped into the
 * diagonal (atilde_ii += a_ik); a row with atilde_ii = 0 interpolates from
 * nothing.  Truncation keeps the pmax largest |w| (ties: lower column) and
 * rescales them by (sum of all w) / (sum of kept w) when that sum is nonzero.
 *
 * Evaluation order: d_k adds over row k in ascending column; atilde_ii starts
 * at a_ii and adds, over row i in ascending column, a_in (weak, not in Chat)
 * or (a_ik*abar_ki)/d_k (strong F); the numerator of j starts at a_ij and adds
 * (a_ik*abar_kj)/d_k over k in F_i^s ascending, skipping terms with
 * abar_kj = 0 or d_k = 0; w = -num/atilde; the sums for the rescaling run in
 * ascending column.
 * Writes up to the returned count of (coarse column, weight) pairs.
 */
static int exti_row(int i, const int *rp, const int *ci, const double *v,
                    const unsigned char *s, const int *cf, const int *cidx, int pmax,
                    exti_ws *ws, int *ocol, double *oval, double *dk_buf)
{
    if (cf[i] == 1) {
        if (ocol) { ocol[0] = cidx[i]; oval[0] = 1.0; }
        return 1;
    }
    int nh = 0;
    int stamp = i + 1;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int j = ci[e];
        if (!s[e]) continue;
        if (cf[j] == 1) {
            if (ws->mark[j] != stamp) { ws->mark[j] = stamp; ws->hat[nh++] = j; }
        } else {
            for (int f = rp[j]; f < rp[j + 1]; ++f) {
                int l = ci[f];
                if (s[f] && cf[l] == 1 && ws->mark[l] != stamp) { ws->mark[l] = stamp; ws->hat[nh++] = l; }
            }
        }
    }
    if (nh == 0) return 0;
    /* sort Chat ascending */
    for (int p = 1; p < nh; ++p) {
        int t = ws->hat[p], q = p - 1;
        while (q >= 0 && ws->hat[q] > t) { ws->hat[q + 1] = ws->hat[q]; --q; }
        ws->hat[q + 1] = t;
    }
    double aii = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) if (ci[e] == i) aii = v[e];
    /* d_k for each strong F neighbour, in row order */
    int nk = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int k = ci[e];
        if (!s[e] || cf[k] == 1) continue;
        double akk = 0.0;
        for (int f = rp[k]; f < rp[k + 1]; ++f) if (ci[f] == k) akk = v[f];
        double d = 0.0;
        for (int f = rp[k]; f < rp[k + 1]; ++f) {
            int l = ci[f];
            if (l == i || (l != k && ws->mark[l] == stamp && cf[l] == 1)) {
                double ab = abar(akk, v[f]);
                if (ab != 0.0) d = d + ab;
            }
        }
        dk_buf[nk++] = d;
    }
    double at = aii;
    nk = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int nn = ci[e];
        if (nn == i) continue;
        if (s[e] && cf[nn] == 0) {
            double d = dk_buf[nk++];
            if (d != 0.0) {
                double akk = 0.0, aki = 0.0;
                for (int f = rp[nn]; f < rp[nn + 1]; ++f) {
                    if (ci[f] == nn) akk = v[f];
                    if (ci[f] == i) aki = v[f];
                }
                double ab = abar(akk, aki);
                if (ab != 0.0) at = at + (v[e] * ab) / d;
            } else {
                at = at + v[e];
            }
        } else if (!s[e] && !(ws->mark[nn] == stamp && cf[nn] == 1)) {
            at = at + v[e];
        }
    }
    if (at == 0.0) return 0;
    for (int p = 0; p < nh; ++p) {
        int j = ws->hat[p];
        double num = 0.0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) if (ci[e] == j) num = v[e];
        nk = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int k = ci[e];
            if (k == i || !s[e] || cf[k] == 1) continue;
            double d = dk_buf[nk++];
            if (d == 0.0) continue;
            double akk = 0.0, akj = 0.0;
            for (int f = rp[k]; f < rp[k + 1]; ++f) {
                if (ci[f] == k) akk = v[f];
                if (ci[f] == j) akj = v[f];
            }
            double ab = abar(akk, akj);
            if (ab == 0.0) continue;
            num = num + (v[e] * ab) / d;
        }
        ws->w[p] = -num / at;
    }
    int keep = nh;
    if (pmax > 0 && nh > pmax) {
        /* choose the pmax largest |w|, ties to the lower column */
        unsigned char *kept = (unsigned char *)calloc(nh, 1);
        for (int q = 0; q < pmax; ++q) {
            int best = -1;
            for (int p = 0; p < nh; ++p) {
                if (kept[p]) continue;
                if (best < 0 || fabs(ws->w[p]) > fabs(ws->w[best])) best = p;
            }
            kept[best] = 1;
        }
        double sall = 0.0, skept = 0.0;
        for (int p = 0; p < nh; ++p) sall = sall + ws->w[p];
        for (int p = 0; p < nh; ++p) if (kept[p]) skept = skept + ws->w[p];
        double scale = (skept != 0.0) ? sall / skept : 1.0;
        int q = 0;
        for (int p = 0; p < nh; ++p) {
            if (!kept[p]) continue;
            ws->hat[q] = ws->hat[p];
            ws->w[q] = (skept != 0.0) ? ws->w[p] * scale : ws->w[p];
            q++;
        }
        free(kept);
        keep = pmax;
    }
    if (ocol)
        for (int p = 0; p < keep; ++p) { ocol[p] = cidx[ws->hat[p]]; oval[p] = ws->w[p]; }
    return keep;
}

static void exti_ws_init(exti_ws *ws, int n, const int *rp)
{
    int maxrow = 1;
    for (int i = 0; i < n; ++i) if (rp[i + 1] - rp[i] > maxrow) maxrow = rp[i + 1] - rp[i];
    ws->cap = maxrow * maxrow + 1;
    ws->mark = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) ws->mark[i] = 0;
    ws->hat = (int *)malloc(sizeof(int) * ws->cap);
    ws->w = (double *)malloc(sizeof(double) * ws->cap);
}

static void exti_ws_free(exti_ws *ws) { free(ws->mark); free(ws->hat); free(ws->w); }

/* row sizes of P (prp[0..n]); returns nnz(P) */
int orc_exti_count(int n, const int *rp, const int *ci, const double *v, const unsigned char *s,
                   const int *cf, int pmax, int *prp)
{
    exti_ws ws; exti_ws_init(&ws, n, rp);
    double *dk = (double *)malloc(sizeof(double) * (ws.cap + 1));
    int *cidx = (int *)calloc(n > 0 ? n : 1, sizeof(int));
    prp[0] = 0;
    for (int i = 0; i < n; ++i) prp[i + 1] = prp[i] + exti_row(i, rp, ci, v, s, cf, cidx, pmax, &ws, NULL, NULL, dk);
    free(dk); free(cidx); exti_ws_free(&ws);
    return prp[n];
}

/* fill P (columns are coarse indices: cidx[j] = number of C points before j) */
void orc_exti_fill(int n, const int *rp, const int *ci, const double *v, const unsigned char *s,
                   const int *cf, int pmax, const int *prp, int *pci, double *pv)
{
    exti_ws ws; exti_ws_init(&ws, n, rp);
    double *dk = (double *)malloc(sizeof(double) * (ws.cap + 1));
    int *cidx = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    int c = 0;
    for (int i = 0; i < n; ++i) { cidx[i] = c; c += (cf[i] == 1); }
    for (int i = 0; i < n; ++i) exti_row(i, rp, ci, v, s, cf, cidx, pmax, &ws, pci + prp[i], pv + prp[i], dk);
    free(dk); free(cidx); exti_ws_free(&ws);
}

/* ------------------------------------------------------------------------ */
/* block ILU(0) and block Jacobi on the scaled matrix  (Eqs. CPRM1 ff.,      */
/* CPTR3M3: the last stage ilu(Abar); remark on block-ILU variants)          */
/* ------------------------------------------------------------------------ */

/*
 * Block ILU(0) in the elimination order given by rank[] (rank[i] = position
 * of cell i).  Textbook IKJ form restricted to the pattern of Abar:
 *   for rows i in increasing rank:
 *     for k in row i with rank[k] < rank[i], increasing rank[k]:
 *       F_ik = F_ik * inv(F_kk)
 *       for j in row i with rank[j] > rank[k] and (k, j) stored: F_ij -= F_ik F_kj
 * F starts as a copy of Abar; on return the lower positions hold L (unit lower
 * factor, identity diagonal implied) and the diagonal and upper positions
 * hold U.  dinv receives inv(U_ii).  Returns 0 or -(1+cell) for a singular
 * pivot block.
 */
int orc_bilu0_factor(int n, int b, const int *rp, const int *ci, const double *Abar,
                     const int *rank, double *F, double *dinv)
{
    size_t bb = (size_t)b * b;
    memcpy(F, Abar, sizeof(double) * bb * rp[n]);
    int *order = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) order[rank[i]] = i;
    int maxrow = 1;
    for (int i = 0; i < n; ++i) if (rp[i + 1] - rp[i] > maxrow) maxrow = rp[i + 1] - rp[i];
    int *low = (int *)malloc(sizeof(int) * maxrow);
    double *tmp = (double *)malloc(sizeof(double) * bb), *work = (double *)malloc(sizeof(double) * bb);
    int rc = 0;
    for (int q = 0; q < n && rc == 0; ++q) {
        int i = order[q];
        int nl = 0;
        for (int e = rp[i]; e < rp[i + 1]; ++e) if (rank[ci[e]] < rank[i]) low[nl++] = e;
        for (int p = 1; p < nl; ++p) {   /* sort lower entries by rank */
            int t = low[p], r = p - 1;
            while (r >= 0 && rank[ci[low[r]]] > rank[ci[t]]) { low[r + 1] = low[r]; --r; }
            low[r + 1] = t;
        }
        for (int p = 0; p < nl; ++p) {
            int e = low[p], k = ci[e];
            block_mul(b, F + e * bb, dinv + (size_t)k * bb, tmp);
            memcpy(F + e * bb, tmp, sizeof(double) * bb);
            for (int f = rp[i]; f < rp[i + 1]; ++f) {
                int j = ci[f];
                if (rank[j] <= rank[k]) continue;
                int g = -1;
                for (int h = rp[k]; h < rp[k + 1]; ++h) if (ci[h] == j) { g = h; break; }
                if (g < 0) continue;
                block_mul(b, F + e * bb, F + g * bb, tmp);
                for (size_t t = 0; t < bb; ++t) F[f * bb + t] = F[f * bb + t] - tmp[t];
            }
        }
        int d = find_diag(rp, ci, i);
        if (d < 0 || block_inverse(b, F + d * bb, dinv + (size_t)i * bb, work) != 0) rc = -(1 + i);
    }
    free(order); free(low); free(tmp); free(work);
    return rc;
}

/* Solve L U w = u with the factors of orc_bilu0_factor:
 * forward  y_i = u_i - sum_{rank k < rank i} L_ik y_k   (increasing rank)
 * backward w_i = inv(U_ii) (y_i - sum_{rank j > rank i} U_ij w_j)  (decreasing rank) */
void orc_bilu0_solve(int n, int b, const int *rp, const int *ci, const double *F,
                     const double *dinv, const int *rank, const double *u, double *w)
{
    size_t bb = (size_t)b * b;
    int *order = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) order[rank[i]] = i;
    double *y = (double *)malloc(sizeof(double) * (size_t)n * b);
    double t[64];
    for (int q = 0; q < n; ++q) {
        int i = order[q];
        for (int r = 0; r < b; ++r) t[r] = u[(size_t)i * b + r];
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int k = ci[e];
            if (rank[k] >= rank[i]) continue;
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < b; ++c) t[r] = t[r] - F[e * bb + r * b + c] * y[(size_t)k * b + c];
        }
        for (int r = 0; r < b; ++r) y[(size_t)i * b + r] = t[r];
    }
    for (int q = n - 1; q >= 0; --q) {
        int i = order[q];
        for (int r = 0; r < b; ++r) t[r] = y[(size_t)i * b + r];
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            int j = ci[e];
            if (rank[j] <= rank[i]) continue;
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < b; ++c) t[r] = t[r] - F[e * bb + r * b + c] * w[(size_t)j * b + c];
        }
        const double *D = dinv + (size_t)i * bb;
        for (int r = 0; r < b; ++r) {
            double s = 0.0;
            for (int c = 0; c < b; ++c) s = s + D[r * b + c] * t[c];
            w[(size_t)i * b + r] = s;
        }
    }
    free(order); free(y);
}

/* block Jacobi: dinv_i = inv(Abar_ii) */
int orc_bjacobi_factor(int n, int b, const int *rp, const int *ci, const double *Abar, double *dinv)
{
    size_t bb = (size_t)b * b;
    double *work = (double *)malloc(sizeof(double) * bb);
    int rc = 0;
    for (int i = 0; i < n && rc == 0; ++i) {
        int d = find_diag(rp, ci, i);
        if (d < 0 || block_inverse(b, Abar + d * bb, dinv + (size_t)i * bb, work) != 0) rc = -(1 + i);
    }
    free(work);
    return rc;
}

/* w_i = dinv_i u_i */
void orc_block_diag_apply(int n, int b, const double *dinv, const double *u, double *w)
{
    size_t bb = (size_t)b * b;
    for (int i = 0; i < n; ++i)
        for (int r = 0; r < b; ++r) {
            double s = 0.0;
            for (int c = 0; c < b; ++c) s = s + dinv[i * bb + r * b + c] * u[(size_t)i * b + c];
            w[(size_t)i * b + r] = s;
        }
}
