// AMG setup on the GPU for the scalar subsystems C_TT and B_PP (the amg(.)
// sub-solver of Eqs. CPTR3M1 and CPTRM2; the paper uses classical
// Ruge-Stueben AMG, this library uses its parallel counterparts):
//   strength of connection -> PMIS coarsening (De Sterck, Yang & Heys 2006)
//   -> extended+i interpolation with truncation (De Sterck, Falgout, Nolting
//   & Yang 2008) -> R = P^T -> Galerkin A_c = R (A P) by SpGEMM -> dense
//   inverse of the coarsest operator.
// Built with floating-point contraction off and with every sum taken in a
// fixed, stated order, so a hierarchy is a deterministic function of its input
// (one thread owns each row; no floating-point atomics anywhere).
#include "internal.h"

#include <algorithm>

namespace cptr {

static inline int blocks_for(long n, int t) { return (int)((n + t - 1) / t > 0 ? (n + t - 1) / t : 1); }

// --------------------------------------------------------------------------
// strength: sigma_i = -1 if a_ii < 0 else +1, m_i = max_{k!=i} (-sigma_i a_ik);
// j != i strong iff m_i > 0 and -sigma_i a_ij >= theta * m_i
// --------------------------------------------------------------------------
__global__ void k_strength(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ v, double theta, unsigned char *__restrict__ s) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = rp[i], b = rp[i + 1];
    double aii = 0.0;
    for (int e = a; e < b; ++e) if (ci[e] == i) aii = v[e];
    const double sg = (aii < 0.0) ? -1.0 : 1.0;
    double m = 0.0;
    bool any = false;
    for (int e = a; e < b; ++e) {
        if (ci[e] == i) continue;
        double t = -sg * v[e];
        if (!any || t > m) { m = t; any = true; }
    }
    const double thr = theta * m;
    for (int e = a; e < b; ++e) {
        unsigned char st = 0;
        if (ci[e] != i && any && m > 0.0 && -sg * v[e] >= thr) st = 1;
        s[e] = st;
    }
}

void amg_strength(int n, const int *rp, const int *ci, const double *v, double theta, unsigned char *s,
                  hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_strength, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, rp, ci, v, theta, s);
    CPTR_CHECK_LAUNCH();
}

// --------------------------------------------------------------------------
// PMIS
// --------------------------------------------------------------------------
// SplitMix64 (Steele, Lea & Flood 2014): output function on seed + (i+1) * gamma
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// measure lambda = |S^T| + random in [0,1): lexicographic (|S^T|, random), then lower index
__device__ inline bool beats(int i, int j, const int *cntT, const uint64_t *h) {
    int ci_ = cntT[i], cj = cntT[j];
    if (ci_ != cj) return ci_ > cj;
    uint64_t hi = h[i], hj = h[j];
    if (hi != hj) return hi > hj;
    return i < j;
}

constexpr int ST_UND = -1, ST_F = 0, ST_C = 1;

// one atomic per wavefront for a count over its lanes
__device__ inline void wave_count_add(bool pred, int *counter) {
    const unsigned long long m = __ballot(pred);
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(counter, (int)__popcll(m));
}

__global__ void k_pmis_init(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                            const unsigned char *__restrict__ s, const int *__restrict__ tpos, uint64_t seed,
                            int *__restrict__ cntT, uint64_t *__restrict__ h, int *__restrict__ state, int *und) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = 0;
    if (i < n) {
        for (int e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] != i && tpos[e] >= 0 && s[tpos[e]]) c++;   // entry (j, i) strong: i in S_j
        cntT[i] = c;
        h[i] = splitmix64(seed, (uint64_t)i);
        state[i] = (c == 0) ? ST_F : ST_UND;
    }
    wave_count_add(i < n && c != 0, und);
}

void amg_pmis_init(int n, const int *rp, const int *ci, const unsigned char *s, const int *tpos, uint64_t seed,
                   int *cntT, uint64_t *h, int *state, int *und, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_pmis_init, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, rp, ci, s, tpos, seed, cntT, h,
                       state, und);
    CPTR_CHECK_LAUNCH();
}

// an undecided point becomes C when it beats every undecided point of its
// symmetrised strong neighbourhood S_i u S^T_i
__global__ void k_pmis_select(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                              const unsigned char *__restrict__ s, const int *__restrict__ tpos,
                              const int *__restrict__ cntT, const uint64_t *__restrict__ h,
                              const int *__restrict__ state, unsigned char *__restrict__ newc) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    unsigned char win = 0;
    if (state[i] == ST_UND) {
        win = 1;
        for (int e = rp[i]; e < rp[i + 1] && win; ++e) {
            int j = ci[e];
            if (j == i) continue;
            bool sym = s[e] || (tpos[e] >= 0 && s[tpos[e]]);
            if (sym && state[j] == ST_UND && !beats(i, j, cntT, h)) win = 0;
        }
    }
    newc[i] = win;
}

// new C points are fixed; undecided points that strongly depend on one become F
__global__ void k_pmis_apply(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                             const unsigned char *__restrict__ s, const unsigned char *__restrict__ newc,
                             int *__restrict__ state, int *und) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool still = false;
    if (i < n && state[i] == ST_UND) {
        if (newc[i]) {
            state[i] = ST_C;
        } else {
            bool f = false;
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                if (s[e] && newc[ci[e]]) { f = true; break; }
            if (f) state[i] = ST_F;
            else still = true;
        }
    }
    wave_count_add(still, und);
}

void amg_pmis_round(int n, const int *rp, const int *ci, const unsigned char *s, const int *tpos, const int *cntT,
                    const uint64_t *h, int *state, unsigned char *newc, int *und, hipStream_t st) {
    hipLaunchKernelGGL(k_pmis_select, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, rp, ci, s, tpos, cntT, h,
                       state, newc);
    hipLaunchKernelGGL(k_pmis_apply, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, rp, ci, s, newc, state, und);
    CPTR_CHECK_LAUNCH();
}

// --------------------------------------------------------------------------
// extended+i interpolation
// --------------------------------------------------------------------------
// upper bound of |Chat_i| (with repeats): C rows 1; F rows: strong C
// neighbours + strong C neighbours of strong F neighbours
__global__ void k_exti_bound(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                             const unsigned char *__restrict__ s, const int *__restrict__ cf, int *__restrict__ ub) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (cf[i] == ST_C) { ub[i] = 1; return; }
    int c = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        if (!s[e]) continue;
        int j = ci[e];
        if (cf[j] == ST_C) { c++; continue; }
        for (int f = rp[j]; f < rp[j + 1]; ++f)
            if (s[f] && cf[ci[f]] == ST_C) c++;
    }
    ub[i] = c > 0 ? c : 1;
}

// the same count, one wavefront per row (coarse levels with long rows): the
// lanes scan each strong F neighbour's row
__global__ void __launch_bounds__(64) k_exti_bound_wave(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const unsigned char *__restrict__ s,
                                                        const int *__restrict__ cf, int *__restrict__ ub) {
    const int i = blockIdx.x, lane = threadIdx.x;
    if (i >= n) return;
    if (cf[i] == ST_C) {
        if (lane == 0) ub[i] = 1;
        return;
    }
    int c = 0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        if (!s[e]) continue;
        const int j = ci[e];
        if (cf[j] == ST_C) { c += (lane == 0); continue; }
        for (int f = rp[j] + lane; f < rp[j + 1]; f += 64)
            if (s[f] && cf[ci[f]] == ST_C) c++;
    }
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane == 0) ub[i] = c > 0 ? c : 1;
}

void amg_exti_bound(int n, const int *rp, const int *ci, const unsigned char *s, const int *cf, int *ub, bool wave,
                    hipStream_t st) {
    if (n == 0) return;
    if (wave)
        hipLaunchKernelGGL(k_exti_bound_wave, dim3(n), dim3(64), 0, st, n, rp, ci, s, cf, ub);
    else
        hipLaunchKernelGGL(k_exti_bound, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, rp, ci, s, cf, ub);
    CPTR_CHECK_LAUNCH();
}

__device__ inline double abar_of(double akk, double akl) {
    return ((akk > 0.0 && akl < 0.0) || (akk < 0.0 && akl > 0.0)) ? akl : 0.0;
}

// value of entry (row, col) of a CSR matrix with ascending columns (0 if absent)
__device__ inline double csr_value(const int *rp, const int *ci, const double *v, int row, int col) {
    int lo = rp[row], hi = rp[row + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int c = ci[mid];
        if (c == col) return v[mid];
        if (c < col) lo = mid + 1; else hi = mid - 1;
    }
    return 0.0;
}

// position of key in a sorted strided array, -1 if absent
__device__ inline int find_sorted(const int *a, int stride, int len, int key) {
    int lo = 0, hi = len - 1;
    while (lo <= hi) {
        int mid = (lo + hi) >> 1;
        int c = a[mid * stride];
        if (c == key) return mid;
        if (c < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

__device__ inline bool in_sorted(const int *a, int stride, int len, int key) {
    return find_sorted(a, stride, len, key) >= 0;
}

// One thread per row.  Writes the row of P (coarse columns, weights) into the
// scratch segment [off[i], off[i] + cnt[i]).  Evaluation order:
//   d_k      = sum over row k ascending of abar_kl, l in Chat_i u {i} (zero terms skipped)
//   atilde   = a_ii, then over row i ascending: + a_in (weak, not in Chat) or
//              + (a_ik abar_ki) / d_k (strong F with d_k != 0) or + a_ik (strong F, d_k = 0)
//   num_j    = a_ij, then over strong F k ascending: + (a_ik abar_kj) / d_k
//   w_ij     = -num_j / atilde
//   truncation to the pmax largest |w| (ties: lower column), kept weights times
//   (sum of all w) / (sum of kept w), both sums in ascending column order.
// The interpolatory set lives in LDS (interleaved across the block) when its
// bound fits EXT_CAP entries, else in the row's global scratch segment.
constexpr int EXT_T = 128;
constexpr int EXT_CAP = 32;

__device__ inline void exti_row(int i, const int *__restrict__ rp, const int *__restrict__ ci,
                                const double *__restrict__ v, const unsigned char *__restrict__ s,
                                const int *__restrict__ cf, const int *__restrict__ cidx,
                                const double *__restrict__ dg, int pmax, int *hat, int hs, double *w,
                                double *__restrict__ td, int *ocol, int *cnt) {
    const int a = rp[i], b = rp[i + 1];
    // gather Chat_i (fine indices), sort, unique
    int nh = 0;
    for (int e = a; e < b; ++e) {
        if (!s[e]) continue;
        int j = ci[e];
        if (cf[j] == ST_C) { hat[(nh++) * hs] = j; continue; }
        for (int f = rp[j]; f < rp[j + 1]; ++f)
            if (s[f] && cf[ci[f]] == ST_C) hat[(nh++) * hs] = ci[f];
    }
    if (nh == 0) { cnt[i] = 0; return; }
    for (int p = 1; p < nh; ++p) {
        int t = hat[p * hs], q = p - 1;
        while (q >= 0 && hat[q * hs] > t) { hat[(q + 1) * hs] = hat[q * hs]; --q; }
        hat[(q + 1) * hs] = t;
    }
    int u = 1;
    for (int p = 1; p < nh; ++p)
        if (hat[p * hs] != hat[(u - 1) * hs]) hat[(u++) * hs] = hat[p * hs];
    nh = u;
    // d_k of every strong F neighbour, stored at the neighbour's entry position
    for (int e = a; e < b; ++e) {
        int k = ci[e];
        if (!s[e] || cf[k] == ST_C) continue;
        const double akk = dg[k];
        double d = 0.0;
        for (int f = rp[k]; f < rp[k + 1]; ++f) {
            int l = ci[f];
            if (l == i || (l != k && cf[l] == ST_C && in_sorted(hat, hs, nh, l))) {
                double ab = abar_of(akk, v[f]);
                if (ab != 0.0) d = d + ab;
            }
        }
        td[e] = d;
    }
    const double aii = dg[i];
    double at = aii;
    for (int e = a; e < b; ++e) {
        int nn = ci[e];
        if (nn == i) continue;
        if (s[e] && cf[nn] == ST_F) {
            double d = td[e];
            if (d != 0.0) {
                double ab = abar_of(dg[nn], csr_value(rp, ci, v, nn, i));
                if (ab != 0.0) at = at + (v[e] * ab) / d;
            } else {
                at = at + v[e];
            }
        } else if (!s[e] && !(cf[nn] == ST_C && in_sorted(hat, hs, nh, nn))) {
            at = at + v[e];
        }
    }
    if (at == 0.0) { cnt[i] = 0; return; }
    // numerators, accumulated in w: a_ij first, then the strong F neighbours'
    // terms in row order (each row k scattered to the positions of its
    // interpolatory columns, so every num_j sees its terms in that order)
    for (int p = 0; p < nh; ++p) w[p] = 0.0;
    for (int e = a; e < b; ++e) {
        const int pos = find_sorted(hat, hs, nh, ci[e]);
        if (pos >= 0) w[pos] = v[e];
    }
    for (int e = a; e < b; ++e) {
        const int k = ci[e];
        if (k == i || !s[e] || cf[k] == ST_C) continue;
        const double d = td[e];
        if (d == 0.0) continue;
        const double akk = dg[k], aik = v[e];
        for (int f = rp[k]; f < rp[k + 1]; ++f) {
            const int pos = find_sorted(hat, hs, nh, ci[f]);
            if (pos < 0) continue;
            const double ab = abar_of(akk, v[f]);
            if (ab == 0.0) continue;
            w[pos] = w[pos] + (aik * ab) / d;
        }
    }
    for (int p = 0; p < nh; ++p) w[p] = -w[p] / at;
    int keep = nh;
    if (pmax > 0 && nh > pmax) {
        // mark kept entries by encoding the column as -1 - col
        for (int q = 0; q < pmax; ++q) {
            int best = -1;
            double bv = 0.0;
            for (int p = 0; p < nh; ++p) {
                if (hat[p * hs] < 0) continue;
                double av = fabs(w[p]);
                if (best < 0 || av > bv) { best = p; bv = av; }
            }
            hat[best * hs] = -1 - hat[best * hs];
        }
        double sall = 0.0, skept = 0.0;
        for (int p = 0; p < nh; ++p) sall = sall + w[p];
        for (int p = 0; p < nh; ++p) if (hat[p * hs] < 0) skept = skept + w[p];
        const double scale = (skept != 0.0) ? sall / skept : 1.0;
        int q = 0;
        for (int p = 0; p < nh; ++p) {
            if (hat[p * hs] >= 0) continue;
            int col = -1 - hat[p * hs];
            double wv = (skept != 0.0) ? w[p] * scale : w[p];
            hat[q * hs] = col;
            w[q] = wv;
            q++;
        }
        keep = pmax;
    }
    for (int p = 0; p < keep; ++p) ocol[p] = cidx[hat[p * hs]];
    cnt[i] = keep;
}

__global__ void __launch_bounds__(EXT_T) k_exti_compute(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                        const double *__restrict__ v,
                                                        const unsigned char *__restrict__ s,
                                                        const int *__restrict__ cf, const int *__restrict__ cidx,
                                                        const double *__restrict__ dg, int pmax,
                                                        const int *__restrict__ off, int *__restrict__ tcol,
                                                        double *__restrict__ tw, double *__restrict__ td,
                                                        int *__restrict__ cnt) {
    __shared__ int shat[EXT_CAP * EXT_T];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int *ocol = tcol + off[i];
    double *w = tw + off[i];
    if (cf[i] == ST_C) {
        ocol[0] = cidx[i];
        w[0] = 1.0;
        cnt[i] = 1;
        return;
    }
    const int ub = off[i + 1] - off[i];
    if (ub <= EXT_CAP)
        exti_row(i, rp, ci, v, s, cf, cidx, dg, pmax, shat + threadIdx.x, EXT_T, w, td, ocol, cnt);
    else
        exti_row(i, rp, ci, v, s, cf, cidx, dg, pmax, ocol, 1, w, td, ocol, cnt);
}

// One wavefront per row for coarse levels (long rows).  Same definition and
// evaluation order as exti_row: the candidate set is expanded and stably
// ranked in LDS, d_k is computed per strong F neighbour by one lane each (row
// k in ascending order), atilde is summed by one lane over row i in ascending
// order, each numerator by one lane over the strong F neighbours in row order,
// and the truncation picks the largest |w| (ties: lower column) round by
// round.  Rows beyond the LDS capacities fall back to exti_row on lane 0.
constexpr int EXW_CAP = 1024;
constexpr int EXW_ROW = 256;

__global__ void __launch_bounds__(64) k_exti_wave(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                  const double *__restrict__ v, const unsigned char *__restrict__ s,
                                                  const int *__restrict__ cf, const int *__restrict__ cidx,
                                                  const double *__restrict__ dg, int pmax,
                                                  const int *__restrict__ off, int *__restrict__ tcol,
                                                  double *__restrict__ tw, double *__restrict__ td,
                                                  int *__restrict__ cnt) {
    __shared__ int cand[EXW_CAP];
    __shared__ int hat[EXW_CAP];
    __shared__ double w[EXW_CAP];
    __shared__ double dk[EXW_ROW];
    __shared__ double term[EXW_ROW];
    __shared__ unsigned char use[EXW_ROW];
    __shared__ unsigned char kept[EXW_CAP];
    __shared__ double at_s;
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    if (i >= n) return;
    int *ocol = tcol + off[i];
    double *ow = tw + off[i];
    if (cf[i] == ST_C) {
        if (lane == 0) { ocol[0] = cidx[i]; ow[0] = 1.0; cnt[i] = 1; }
        return;
    }
    const int a = rp[i], b = rp[i + 1];
    const int ub = off[i + 1] - off[i];
    if (ub > EXW_CAP || b - a > EXW_ROW) {
        if (lane == 0) exti_row(i, rp, ci, v, s, cf, cidx, dg, pmax, ocol, 1, ow, td, ocol, cnt);
        return;
    }
    // 1. candidates with repeats, in row order
    int nc = 0;
    for (int e = a; e < b; ++e) {
        if (!s[e]) continue;
        const int j = ci[e];
        if (cf[j] == ST_C) {
            if (lane == 0) cand[nc] = j;
            nc += 1;
            continue;
        }
        const int f0 = rp[j], len = rp[j + 1] - f0;
        for (int q0 = 0; q0 < len; q0 += 64) {
            const int f = f0 + q0 + lane;
            const bool take = (q0 + lane < len) && s[f] && cf[ci[f]] == ST_C;
            const unsigned long long mask = __ballot(take);
            if (take) cand[nc + __popcll(mask & ((1ull << lane) - 1ull))] = ci[f];
            nc += __popcll(mask);
        }
    }
    __syncthreads();
    if (nc == 0) {
        if (lane == 0) cnt[i] = 0;
        return;
    }
    // 2. sort (bitonic network, padded to a power of two) + unique
    int S = 1;
    while (S < nc) S <<= 1;
    for (int p = nc + lane; p < S; p += 64) cand[p] = 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= S; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < S; t += 64) {
                const int q = t ^ j;
                if (q > t) {
                    const int x = cand[t], y = cand[q];
                    if ((x > y) == ((t & k) == 0)) { cand[t] = y; cand[q] = x; }
                }
            }
            __syncthreads();
        }
    }
    int nh = 0;
    for (int c0 = 0; c0 < nc; c0 += 64) {
        const int p = c0 + lane;
        const bool head = p < nc && (p == 0 || cand[p] != cand[p - 1]);
        const unsigned long long mask = __ballot(head);
        if (head) hat[nh + __popcll(mask & ((1ull << lane) - 1ull))] = cand[p];
        nh += __popcll(mask);
    }
    __syncthreads();
    auto inhat = [&](int key) {
        int lo = 0, hi = nh - 1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const int c = hat[mid];
            if (c == key) return true;
            if (c < key) lo = mid + 1; else hi = mid - 1;
        }
        return false;
    };
    // 3. d_k per strong F neighbour (one lane per entry, row k ascending)
    for (int e = a + lane; e < b; e += 64) {
        const int k = ci[e];
        double d = 0.0;
        if (s[e] && cf[k] != ST_C) {
            const double akk = dg[k];
            for (int f = rp[k]; f < rp[k + 1]; ++f) {
                const int l = ci[f];
                if (l == i || (l != k && cf[l] == ST_C && inhat(l))) {
                    const double ab = abar_of(akk, v[f]);
                    if (ab != 0.0) d = d + ab;
                }
            }
        }
        dk[e - a] = d;
        td[e] = d;
    }
    __syncthreads();
    // 4. terms of atilde, summed in row order by lane 0
    for (int e = a + lane; e < b; e += 64) {
        const int nn = ci[e];
        unsigned char u = 0;
        double t = 0.0;
        if (nn != i) {
            if (s[e] && cf[nn] == ST_F) {
                const double d = dk[e - a];
                if (d != 0.0) {
                    const double ab = abar_of(dg[nn], csr_value(rp, ci, v, nn, i));
                    if (ab != 0.0) { t = (v[e] * ab) / d; u = 1; }
                } else {
                    t = v[e];
                    u = 1;
                }
            } else if (!s[e] && !(cf[nn] == ST_C && inhat(nn))) {
                t = v[e];
                u = 1;
            }
        }
        term[e - a] = t;
        use[e - a] = u;
    }
    __syncthreads();
    if (lane == 0) {
        double at = dg[i];
        for (int e = 0; e < b - a; ++e)
            if (use[e]) at = at + term[e];
        at_s = at;
    }
    __syncthreads();
    const double at = at_s;
    if (at == 0.0) {
        if (lane == 0) cnt[i] = 0;
        return;
    }
    // 5. weights.  The numerators accumulate in w: a_ij first, then the
    // strong F neighbours in row order, the lanes splitting each row k (its
    // columns are distinct, so no two lanes meet on one numerator)
    for (int p = lane; p < nh; p += 64) {
        w[p] = 0.0;
        kept[p] = 0;
    }
    __syncthreads();
    for (int e = a + lane; e < b; e += 64) {
        const int pos = find_sorted(hat, 1, nh, ci[e]);
        if (pos >= 0) w[pos] = v[e];
    }
    __syncthreads();
    for (int e = a; e < b; ++e) {
        const int k = ci[e];
        if (k == i || !s[e] || cf[k] == ST_C) continue;
        const double d = dk[e - a];
        if (d == 0.0) continue;
        const double akk = dg[k], aik = v[e];
        for (int f = rp[k] + lane; f < rp[k + 1]; f += 64) {
            const int pos = find_sorted(hat, 1, nh, ci[f]);
            if (pos < 0) continue;
            const double ab = abar_of(akk, v[f]);
            if (ab == 0.0) continue;
            w[pos] = w[pos] + (aik * ab) / d;
        }
        __syncthreads();
    }
    for (int p = lane; p < nh; p += 64) w[p] = -w[p] / at;
    __syncthreads();
    int keep = nh;
    if (pmax > 0 && nh > pmax) {
        for (int round = 0; round < pmax; ++round) {
            double bv = -1.0;
            int bp = 0x7fffffff;
            for (int p = lane; p < nh; p += 64) {
                if (kept[p]) continue;
                const double av = fabs(w[p]);
                if (av > bv || (av == bv && p < bp)) { bv = av; bp = p; }
            }
            for (int d = 32; d >= 1; d >>= 1) {
                const double ov = __shfl_xor(bv, d, 64);
                const int op = __shfl_xor(bp, d, 64);
                if (ov > bv || (ov == bv && op < bp)) { bv = ov; bp = op; }
            }
            if (lane == 0) kept[bp] = 1;
            __syncthreads();
        }
        if (lane == 0) {
            double sall = 0.0, skept = 0.0;
            for (int p = 0; p < nh; ++p) sall = sall + w[p];
            for (int p = 0; p < nh; ++p) if (kept[p]) skept = skept + w[p];
            const double scale = (skept != 0.0) ? sall / skept : 1.0;
            int q = 0;
            for (int p = 0; p < nh; ++p) {
                if (!kept[p]) continue;
                ocol[q] = cidx[hat[p]];
                ow[q] = (skept != 0.0) ? w[p] * scale : w[p];
                q++;
            }
            cnt[i] = pmax;
        }
        return;
    }
    for (int p = lane; p < keep; p += 64) {
        ocol[p] = cidx[hat[p]];
        ow[p] = w[p];
    }
    if (lane == 0) cnt[i] = keep;
}

// One group of G lanes per row (64 / G rows per wavefront: 8 lanes on the
// 5-point fine level, 32 or 64 on the Galerkin levels).  The row's entries
// and the rows of its strong F neighbours (flattened into one list, entry t of
// the list belonging to the neighbour whose extent holds t) are fetched into
// LDS by all lanes at once; every quantity of exti_row is then formed from
// LDS with exti_row's definition and summation order:
//   Chat_i  - the distinct candidates (rank of each first occurrence);
//   d_k     - one lane per strong F neighbour, over its extent in order;
//   atilde  - one lane over the row's terms in order;
//   num_j   - a_ij, then the neighbours' terms in list order (= row order of
//             the neighbours, then of their rows), one lane per j;
//   truncation as in exti_row.
// Rows beyond the caps (RCAP entries, WCAP listed entries, HCAP candidates)
// run exti_row on the group's first lane.
template <int G, int RCAP, int WCAP, int HCAP>
__global__ void __launch_bounds__(64) k_exti_group(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                                   const double *__restrict__ v, const unsigned char *__restrict__ s,
                                                   const int *__restrict__ cf, const int *__restrict__ cidx,
                                                   const double *__restrict__ dg, int pmax,
                                                   const int *__restrict__ off, int *__restrict__ tcol,
                                                   double *__restrict__ tw, double *__restrict__ td,
                                                   int *__restrict__ cnt) {
    constexpr int NG = 64 / G;
    constexpr int RPL = (RCAP + G - 1) / G;
    // row entry flags
    constexpr unsigned char RS = 1, RC = 2, RF = 4, RX = 8, RU = 16;
    __shared__ int r_col[NG][RCAP];
    __shared__ double r_val[NG][RCAP];
    __shared__ unsigned char r_fl[NG][RCAP];
    __shared__ int r_beg[NG][RCAP];
    __shared__ int r_off[NG][RCAP + 1];
    __shared__ double r_dg[NG][RCAP];
    __shared__ double r_d[NG][RCAP];
    __shared__ double r_term[NG][RCAP];
    // listed entries: column and value, overwritten in place (same lane) by
    // the numerator position and term
    __shared__ int f_col[NG][WCAP];
    __shared__ double f_val[NG][WCAP];
    __shared__ unsigned char f_fl[NG][WCAP];
    __shared__ int h_cand[NG][HCAP];
    __shared__ unsigned char h_first[NG][HCAP];
    __shared__ int h_hat[NG][HCAP];
    __shared__ double h_w[NG][HCAP];
    __shared__ unsigned char h_kept[NG][HCAP];
    __shared__ double g_at[NG];
    const int lane = threadIdx.x, g = lane / G, gl = lane % G;
    const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (g * G));
    const int i = blockIdx.x * NG + g;
    const bool act = i < n;
    const bool isC = act && cf[i] == ST_C;
    const int a = act ? rp[i] : 0;
    const int L = act ? rp[i + 1] - a : 0;
    const int ub = act ? off[i + 1] - off[i] : 0;
    bool work = act && !isC && L <= RCAP && ub <= HCAP;
    bool fb = act && !isC && !work;
    // A. the row's entries and its neighbours' extents
    int W = 0;
    {
        int lens[RPL];
        int mine = 0;
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
            const int q = gl * RPL + u;
            int len = 0;
            if (work && q < L) {
                const int e = a + q;
                const int col = ci[e];
                const bool sv = s[e] != 0;
                const int c = cf[col];
                unsigned char fl = (sv ? RS : 0) | (c == ST_C ? RC : 0) | (c == ST_F ? RF : 0);
                if (sv && c != ST_C) {
                    fl |= RX;
                    const int b0 = rp[col];
                    len = rp[col + 1] - b0;
                    r_beg[g][q] = b0;
                    r_dg[g][q] = dg[col];
                }
                r_col[g][q] = col;
                r_val[g][q] = v[e];
                r_fl[g][q] = fl;
            }
            lens[u] = len;
            mine += len;
        }
        int incl = mine;
        for (int d = 1; d < G; d <<= 1) {
            const int y = __shfl_up(incl, d, G);
            if (gl >= d) incl += y;
        }
        int run = incl - mine;
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
            const int q = gl * RPL + u;
            if (q < RCAP) r_off[g][q] = run;
            run += lens[u];
        }
        W = __shfl(incl, G - 1, G);
        if (gl == 0) r_off[g][RCAP] = W;
        if (work && W > WCAP) {
            work = false;
            fb = true;
        }
    }
    __syncthreads();
    // B. the flattened rows of the strong F neighbours
    if (work) {
        for (int t = gl; t < W; t += G) {
            int lo = 0, hi = L - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (r_off[g][mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int f = r_beg[g][lo] + (t - r_off[g][lo]);
            const int l = ci[f];
            f_col[g][t] = l;
            f_val[g][t] = v[f];
            f_fl[g][t] = (s[f] ? RS : 0) | (cf[l] == ST_C ? RC : 0);
        }
    }
    __syncthreads();
    // C. candidates with repeats: strong C entries of the row, then strong C
    // entries of the listed rows
    int nc = 0;
    if (work) {
        for (int q0 = 0; q0 < L; q0 += G) {
            const int q = q0 + gl;
            const bool take = q < L && (r_fl[g][q] & (RS | RC)) == (RS | RC);
            const unsigned long long m = __ballot(take) & gmask;
            if (take) h_cand[g][nc + __popcll(m & ((1ull << lane) - 1ull))] = r_col[g][q];
            nc += __popcll(m);
        }
        for (int t0 = 0; t0 < W; t0 += G) {
            const int t = t0 + gl;
            const bool take = t < W && (f_fl[g][t] & (RS | RC)) == (RS | RC);
            const unsigned long long m = __ballot(take) & gmask;
            if (take) h_cand[g][nc + __popcll(m & ((1ull << lane) - 1ull))] = f_col[g][t];
            nc += __popcll(m);
        }
    }
    __syncthreads();
    // D. first occurrences
    if (work) {
        for (int t = gl; t < nc; t += G) {
            const int x = h_cand[g][t];
            bool first = true;
            for (int u = 0; u < t; ++u)
                if (h_cand[g][u] == x) { first = false; break; }
            h_first[g][t] = first ? 1 : 0;
        }
    }
    __syncthreads();
    // E. each distinct candidate at its rank: Chat_i in ascending order
    int nh = 0;
    if (work) {
        int cntf = 0;
        for (int t = gl; t < nc; t += G) {
            if (!h_first[g][t]) continue;
            ++cntf;
            const int x = h_cand[g][t];
            int rank = 0;
            for (int u = 0; u < nc; ++u) rank += (h_first[g][u] && h_cand[g][u] < x) ? 1 : 0;
            h_hat[g][rank] = x;
        }
        for (int d = G >> 1; d >= 1; d >>= 1) cntf += __shfl_xor(cntf, d, G);
        nh = cntf;
    }
    __syncthreads();
    auto hat_pos = [&](int key) {
        int lo = 0, hi = nh - 1;
        while (lo <= hi) {
            const int mid = (lo + hi) >> 1;
            const int c = h_hat[g][mid];
            if (c == key) return mid;
            if (c < key) lo = mid + 1; else hi = mid - 1;
        }
        return -1;
    };
    // F. d_k of every strong F neighbour and the terms of atilde
    if (work && nh > 0) {
        for (int q = gl; q < L; q += G) {
            const unsigned char fl = r_fl[g][q];
            const int col = r_col[g][q];
            double d = 0.0, aki = 0.0;
            if (fl & RX) {
                const double akk = r_dg[g][q];
                for (int t = r_off[g][q]; t < r_off[g][q + 1]; ++t) {
                    const int l = f_col[g][t];
                    if (l == i) aki = f_val[g][t];
                    if (l == i || (l != col && (f_fl[g][t] & RC) && hat_pos(l) >= 0)) {
                        const double ab = abar_of(akk, f_val[g][t]);
                        if (ab != 0.0) d = d + ab;
                    }
                }
            }
            r_d[g][q] = d;
            bool use = false;
            double term = 0.0;
            if (col != i) {
                if ((fl & RS) && (fl & RF)) {
                    if (d != 0.0) {
                        const double ab = abar_of(r_dg[g][q], aki);
                        if (ab != 0.0) { term = (r_val[g][q] * ab) / d; use = true; }
                    } else {
                        term = r_val[g][q];
                        use = true;
                    }
                } else if (!(fl & RS) && !((fl & RC) && hat_pos(col) >= 0)) {
                    term = r_val[g][q];
                    use = true;
                }
            }
            r_term[g][q] = term;
            if (use) r_fl[g][q] = fl | RU;
        }
        for (int p = gl; p < nh; p += G) {
            h_w[g][p] = 0.0;
            h_kept[g][p] = 0;
        }
    }
    __syncthreads();
    // G. atilde (one lane, row order); a_ij into the numerators; the listed
    // entries' numerator terms
    if (work && nh > 0) {
        if (gl == 0) {
            double at = dg[i];
            for (int q = 0; q < L; ++q)
                if (r_fl[g][q] & RU) at = at + r_term[g][q];
            g_at[g] = at;
        }
        for (int q = gl; q < L; q += G) {
            const int pos = hat_pos(r_col[g][q]);
            if (pos >= 0) h_w[g][pos] = r_val[g][q];
        }
        for (int t = gl; t < W; t += G) {
            int lo = 0, hi = L - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (r_off[g][mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int k = r_col[g][lo];
            const double d = r_d[g][lo];
            int pos = -1;
            double con = 0.0;
            if (k != i && d != 0.0) {
                pos = hat_pos(f_col[g][t]);
                if (pos >= 0) {
                    const double ab = abar_of(r_dg[g][lo], f_val[g][t]);
                    if (ab != 0.0) con = (r_val[g][lo] * ab) / d;
                    else pos = -1;
                }
            }
            f_col[g][t] = pos;
            f_val[g][t] = con;
        }
    }
    __syncthreads();
    // H. numerators summed in list order, weights
    double at = 0.0;
    if (work && nh > 0) {
        at = g_at[g];
        if (at != 0.0) {
            for (int p = gl; p < nh; p += G) {
                double num = h_w[g][p];
                for (int t = 0; t < W; ++t)
                    if (f_col[g][t] == p) num = num + f_val[g][t];
                h_w[g][p] = -num / at;
            }
        }
    }
    __syncthreads();
    // I. truncation to the pmax largest |w| (ties: lower position)
    const bool trunc = work && nh > 0 && at != 0.0 && pmax > 0 && nh > pmax;
    for (int round = 0; round < pmax; ++round) {
        if (trunc) {
            double bv = -1.0;
            int bp = 0x7fffffff;
            for (int p = gl; p < nh; p += G) {
                if (h_kept[g][p]) continue;
                const double av = fabs(h_w[g][p]);
                if (av > bv || (av == bv && p < bp)) { bv = av; bp = p; }
            }
            for (int d = G >> 1; d >= 1; d >>= 1) {
                const double ov = __shfl_xor(bv, d, G);
                const int op = __shfl_xor(bp, d, G);
                if (ov > bv || (ov == bv && op < bp)) { bv = ov; bp = op; }
            }
            if (gl == 0) h_kept[g][bp] = 1;
        }
        __syncthreads();
    }
    // J. output
    if (act) {
        int *ocol = tcol + off[i];
        double *ow = tw + off[i];
        if (isC) {
            if (gl == 0) { ocol[0] = cidx[i]; ow[0] = 1.0; cnt[i] = 1; }
        } else if (fb) {
            if (gl == 0) exti_row(i, rp, ci, v, s, cf, cidx, dg, pmax, ocol, 1, ow, td, ocol, cnt);
        } else if (nh == 0 || at == 0.0) {
            if (gl == 0) cnt[i] = 0;
        } else if (trunc) {
            if (gl == 0) {
                double sall = 0.0, skept = 0.0;
                for (int p = 0; p < nh; ++p) sall = sall + h_w[g][p];
                for (int p = 0; p < nh; ++p) if (h_kept[g][p]) skept = skept + h_w[g][p];
                const double scale = (skept != 0.0) ? sall / skept : 1.0;
                int q = 0;
                for (int p = 0; p < nh; ++p) {
                    if (!h_kept[g][p]) continue;
                    ocol[q] = cidx[h_hat[g][p]];
                    ow[q] = (skept != 0.0) ? h_w[g][p] * scale : h_w[g][p];
                    q++;
                }
                cnt[i] = pmax;
            }
        } else {
            for (int p = gl; p < nh; p += G) {
                ocol[p] = cidx[h_hat[g][p]];
                ow[p] = h_w[g][p];
            }
            if (gl == 0) cnt[i] = nh;
        }
    }
}

void amg_exti_compute_group(int n, int lanes, const int *rp, const int *ci, const double *v,
                            const unsigned char *s, const int *cf, const int *cidx, const double *dg, int pmax,
                            const int *off, int *tcol, double *tw, double *td, int *cnt, hipStream_t st) {
    if (n == 0) return;
    if (lanes == 8)
        hipLaunchKernelGGL((k_exti_group<8, 8, 32, 16>), dim3((n + 7) / 8), dim3(64), 0, st, n, rp, ci, v, s, cf,
                           cidx, dg, pmax, off, tcol, tw, td, cnt);
    else if (lanes == 32)
        hipLaunchKernelGGL((k_exti_group<32, 32, 256, 64>), dim3((n + 1) / 2), dim3(64), 0, st, n, rp, ci, v, s, cf,
                           cidx, dg, pmax, off, tcol, tw, td, cnt);
    else
        hipLaunchKernelGGL((k_exti_group<64, 64, 512, 128>), dim3(n), dim3(64), 0, st, n, rp, ci, v, s, cf, cidx,
                           dg, pmax, off, tcol, tw, td, cnt);
    CPTR_CHECK_LAUNCH();
}

void amg_exti_compute_wave(int n, const int *rp, const int *ci, const double *v, const unsigned char *s,
                           const int *cf, const int *cidx, const double *dg, int pmax, const int *off, int *tcol,
                           double *tw, double *td, int *cnt, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_exti_wave, dim3(n), dim3(64), 0, st, n, rp, ci, v, s, cf, cidx, dg, pmax, off, tcol, tw, td,
                       cnt);
    CPTR_CHECK_LAUNCH();
}

void amg_exti_compute2(int n, const int *rp, const int *ci, const double *v, const unsigned char *s, const int *cf,
                       const int *cidx, const double *dg, int pmax, const int *off, int *tcol, double *tw,
                       double *td, int *cnt, hipStream_t st) {
    hipLaunchKernelGGL(k_exti_compute, dim3(blocks_for(n, EXT_T)), dim3(EXT_T), 0, st, n, rp, ci, v, s, cf, cidx, dg,
                       pmax, off, tcol, tw, td, cnt);
    CPTR_CHECK_LAUNCH();
}

// copy segments [off[i], off[i] + (prp[i+1]-prp[i])) to the compact CSR,
// CP_G lanes per row
constexpr int CP_G = 8;

__global__ void k_compact(int n, const int *__restrict__ off, const int *__restrict__ tcol,
                          const double *__restrict__ tw, const int *__restrict__ prp, int *__restrict__ pci,
                          double *__restrict__ pv) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / CP_G), l = (int)(t % CP_G);
    if (i >= n) return;
    const int o = off[i], d = prp[i], c = prp[i + 1] - prp[i];
    for (int p = l; p < c; p += CP_G) {
        pci[d + p] = tcol[o + p];
        pv[d + p] = tw[o + p];
    }
}

void amg_compact(int n, const int *off, const int *tcol, const double *tw, const int *prp, int *pci, double *pv,
                 hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_compact, dim3(blocks_for((size_t)n * CP_G, 256)), dim3(256), 0, st, n, off, tcol, tw, prp,
                       pci, pv);
    CPTR_CHECK_LAUNCH();
}

// --------------------------------------------------------------------------
// transpose (R = P^T): count, scan, scatter (in arbitrary order, with the
// target row of every entry), then every entry moves to its rank in its row
// (the columns of a row are distinct, so the ranks are a permutation)
// --------------------------------------------------------------------------
__global__ void k_tr_count(int nr, const int *__restrict__ rp, const int *__restrict__ ci, int *__restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) atomicAdd(&cnt[ci[e]], 1);
}

__global__ void k_tr_scatter(int nr, const int *__restrict__ rp, const int *__restrict__ ci,
                             const double *__restrict__ v, int *__restrict__ cursor, int *__restrict__ tci,
                             double *__restrict__ tv, int *__restrict__ trow) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nr) return;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int c = ci[e];
        const int p = atomicAdd(&cursor[c], 1);
        tci[p] = i;
        tv[p] = v[e];
        trow[p] = c;
    }
}

// rows longer than this are copied as they are and sorted by k_sort_rows_huge
constexpr int TR_RANK_MAX = 1024;

__global__ void k_tr_rank(int nnz, const int *__restrict__ rpT, const int *__restrict__ trow,
                          const int *__restrict__ tci, const double *__restrict__ tv, int *__restrict__ ciT,
                          double *__restrict__ vT) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nnz) return;
    const int c = trow[t];
    const int a = rpT[c], len = rpT[c + 1] - a;
    const int key = tci[t];
    if (len > TR_RANK_MAX) {
        ciT[t] = key;
        vT[t] = tv[t];
        return;
    }
    int rank = 0;
    for (int q = a; q < a + len; ++q) rank += (tci[q] < key) ? 1 : 0;
    ciT[a + rank] = key;
    vT[a + rank] = tv[t];
}

// one thread per row: insertion sort in place of the rows beyond TR_RANK_MAX
__global__ void k_sort_rows_huge(int n, const int *__restrict__ rp, int *__restrict__ ci, double *__restrict__ v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int a = rp[i], len = rp[i + 1] - a;
    if (len <= TR_RANK_MAX) return;
    for (int p = a + 1; p < a + len; ++p) {
        const int cc = ci[p];
        const double xx = v[p];
        int q = p - 1;
        while (q >= a && ci[q] > cc) { ci[q + 1] = ci[q]; v[q + 1] = v[q]; --q; }
        ci[q + 1] = cc;
        v[q + 1] = xx;
    }
}

void amg_transpose(int nr, int nc, int nnz, const int *rp, const int *ci, const double *v, int *rpT, int *ciT,
                   double *vT, int *work, hipStream_t st) {
    fill_int(work, 0, (size_t)nc + 1, st);
    hipLaunchKernelGGL(k_tr_count, dim3(blocks_for(nr, 256)), dim3(256), 0, st, nr, rp, ci, work);
    scan_exclusive(work, rpT, nc, nullptr, st);
    if (nnz == 0) return;
    CPTR_HIP(hipMemcpyAsync(work, rpT, sizeof(int) * nc, hipMemcpyDeviceToDevice, st));
    DBuf<int> tci, trow;
    DBuf<double> tv;
    tci.alloc(nnz);
    trow.alloc(nnz);
    tv.alloc(nnz);
    hipLaunchKernelGGL(k_tr_scatter, dim3(blocks_for(nr, 256)), dim3(256), 0, st, nr, rp, ci, v, work, tci.p, tv.p,
                       trow.p);
    hipLaunchKernelGGL(k_tr_rank, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, nnz, rpT, trow.p, tci.p, tv.p, ciT,
                       vT);
    hipLaunchKernelGGL(k_sort_rows_huge, dim3(blocks_for(nc, 256)), dim3(256), 0, st, nc, rpT, ciT, vT);
    CPTR_CHECK_LAUNCH();
}

// --------------------------------------------------------------------------
// SpGEMM C = A B (Gustavson, one thread per row, open-addressing hash
// accumulator processed in A's row order, so every output entry sums its terms
// in ascending k starting from the first term)
// --------------------------------------------------------------------------
// maxprod[1], the shape word, gets bit 0 when some row of A has more than
// SPR_EA entries or reaches a row of B with more than SPR_FB entries: the
// register kernel below takes only products within both
constexpr int SPR_EA = 5, SPR_FB = 4;

__global__ void k_spgemm_bound(int m, const int *__restrict__ arp, const int *__restrict__ aci,
                               const int *__restrict__ brp, int *__restrict__ ub, int *maxprod) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = 0;
    bool wide = false;
    if (i < m) {
        const int e0 = arp[i], e1 = arp[i + 1];
        wide = e1 - e0 > SPR_EA;
        for (int e = e0; e < e1; ++e) {
            const int k = aci[e];
            const int nb = brp[k + 1] - brp[k];
            c += nb;
            wide = wide || nb > SPR_FB;
        }
        ub[i] = 2 * c + 1;      // hash capacity
    }
    if (maxprod) {
        // one atomic of each kind per wavefront
        int w = c;
        for (int d = 32; d >= 1; d >>= 1) w = max(w, __shfl_xor(w, d, 64));
        const bool any_wide = __ballot(wide) != 0;
        if ((threadIdx.x & 63) == 0) {
            atomicMax(maxprod, w);
            if (any_wide) atomicOr(maxprod + 1, 1);
        }
    }
}

void amg_spgemm_bound(int m, const int *arp, const int *aci, const int *brp, int *ub, int *maxprod, hipStream_t st) {
    if (m == 0) return;
    if (maxprod) fill_int(maxprod, 0, 2, st);
    hipLaunchKernelGGL(k_spgemm_bound, dim3(blocks_for(m, 256)), dim3(256), 0, st, m, arp, aci, brp, ub, maxprod);
    CPTR_CHECK_LAUNCH();
}

// One thread per output row.  The accumulator is an open-addressing hash
// table filled strictly in A's row order, so every output entry sums its
// terms in ascending k starting from the first term.  Rows whose table fits
// (capacity <= SPG_CAP) keep it in LDS, interleaved across the block's
// threads; longer rows use their segment of the global scratch.
constexpr int SPG_T = 64;
constexpr int SPG_CAP = 48;

__device__ inline void spgemm_row(int i, const int *__restrict__ arp, const int *__restrict__ aci,
                                  const double *__restrict__ av, const int *__restrict__ brp,
                                  const int *__restrict__ bci, const double *__restrict__ bv, int *hk, double *hv,
                                  int stride, int cap, int *ok, double *ov, int *cnt) {
    for (int p = 0; p < cap; ++p) hk[p * stride] = -1;
    for (int e = arp[i]; e < arp[i + 1]; ++e) {
        const int k = aci[e];
        const double a = av[e];
        for (int f = brp[k]; f < brp[k + 1]; ++f) {
            const int j = bci[f];
            const double t = a * bv[f];
            unsigned hsh = ((unsigned)j * 2654435761u) % (unsigned)cap;
            while (true) {
                const int key = hk[hsh * stride];
                if (key == -1) { hk[hsh * stride] = j; hv[hsh * stride] = t; break; }
                if (key == j) { hv[hsh * stride] = hv[hsh * stride] + t; break; }
                hsh = (hsh + 1 == (unsigned)cap) ? 0u : hsh + 1;
            }
        }
    }
    // compact the occupied slots to the front, sort by column, write out
    int u = 0;
    for (int p = 0; p < cap; ++p) {
        const int c = hk[p * stride];
        if (c < 0) continue;
        const double x = hv[p * stride];
        hk[u * stride] = c;
        hv[u * stride] = x;
        u++;
    }
    for (int p = 1; p < u; ++p) {
        const int c = hk[p * stride];
        const double x = hv[p * stride];
        int q = p - 1;
        while (q >= 0 && hk[q * stride] > c) {
            hk[(q + 1) * stride] = hk[q * stride];
            hv[(q + 1) * stride] = hv[q * stride];
            --q;
        }
        hk[(q + 1) * stride] = c;
        hv[(q + 1) * stride] = x;
    }
    if (ok != hk)
        for (int p = 0; p < u; ++p) { ok[p] = hk[p * stride]; ov[p] = hv[p * stride]; }
    cnt[i] = u;
}

__global__ void __launch_bounds__(SPG_T) k_spgemm_compute(int m, const int *__restrict__ arp,
                                                          const int *__restrict__ aci, const double *__restrict__ av,
                                                          const int *__restrict__ brp, const int *__restrict__ bci,
                                                          const double *__restrict__ bv, const int *__restrict__ off,
                                                          int *__restrict__ tcol, double *__restrict__ tval,
                                                          int *__restrict__ cnt) {
    __shared__ int sk[SPG_CAP * SPG_T];
    __shared__ double sv[SPG_CAP * SPG_T];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int cap = off[i + 1] - off[i];
    int *ok = tcol + off[i];
    double *ov = tval + off[i];
    if (cap <= SPG_CAP)
        spgemm_row(i, arp, aci, av, brp, bci, bv, sk + threadIdx.x, sv + threadIdx.x, SPG_T, cap, ok, ov, cnt);
    else
        spgemm_row(i, arp, aci, av, brp, bci, bv, ok, ov, 1, cap, ok, ov, cnt);
}

// One thread per row for rows of at most EA entries of A whose rows of B
// have at most FB entries (the fine level's A P: five-point rows times
// truncated interpolation rows).  Every product stays in registers, product
// p = (entry e of A's row, entry f of B's row) in A's row order, then B's:
// the first product of a column starts its sum and the later ones are added
// in product order -- the sequential accumulation, bit for bit -- and each
// column's rank among the row's distinct columns places it in the sorted
// output row.  No LDS, so the row's loads are all in flight together.
template <int EA, int FB>
__device__ inline unsigned spr_products(int i, const int *__restrict__ arp, const int *__restrict__ aci,
                                        const double *__restrict__ av, const int *__restrict__ brp,
                                        const int *__restrict__ bci, const double *__restrict__ bv,
                                        int (&col)[EA * FB], double (&t)[EA * FB]) {
    constexpr int NP = EA * FB;
    static_assert(NP <= 32, "first-occurrence mask is 32 bits");
    const int e0 = arp[i], na = arp[i + 1] - e0;
    int kk[EA];
    double a[EA];
#pragma unroll
    for (int e = 0; e < EA; ++e) {
        const bool on = e < na;
        kk[e] = on ? aci[e0 + e] : 0;
        a[e] = on ? av[e0 + e] : 0.0;
    }
    int fb[EA], nb[EA];
#pragma unroll
    for (int e = 0; e < EA; ++e) {
        const bool on = e < na;
        fb[e] = on ? brp[kk[e]] : 0;
        nb[e] = on ? brp[kk[e] + 1] - fb[e] : 0;
    }
#pragma unroll
    for (int e = 0; e < EA; ++e) {
#pragma unroll
        for (int f = 0; f < FB; ++f) {
            const int p = e * FB + f;
            const bool on = f < nb[e];
            col[p] = on ? bci[fb[e] + f] : -1 - p;     // an empty slot: a column of its own, below every real one
            t[p] = on ? a[e] * bv[fb[e] + f] : 0.0;
        }
    }
    // bit p: product p is its column's first
    unsigned first = 0;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        bool fst = col[p] >= 0;
#pragma unroll
        for (int q = 0; q < p; ++q) fst = fst && col[q] != col[p];
        first |= fst ? (1u << p) : 0u;
    }
    return first;
}

// column p's sum over its products in order, and its rank in the row
template <int NP>
__device__ inline double spr_sum(int p, unsigned first, const int (&col)[NP], const double (&t)[NP], int &rank) {
    double s = t[p];
#pragma unroll
    for (int q = p + 1; q < NP; ++q) s = (col[q] == col[p]) ? s + t[q] : s;
    int r = 0;
#pragma unroll
    for (int q = 0; q < NP; ++q) r += (((first >> q) & 1u) && col[q] < col[p]) ? 1 : 0;
    rank = r;
    return s;
}

template <int EA, int FB>
__global__ void __launch_bounds__(256) k_spgemm_reg(int m, const int *__restrict__ arp, const int *__restrict__ aci,
                                                    const double *__restrict__ av, const int *__restrict__ brp,
                                                    const int *__restrict__ bci, const double *__restrict__ bv,
                                                    const int *__restrict__ off, int *__restrict__ tcol,
                                                    double *__restrict__ tval, int *__restrict__ cnt) {
    constexpr int NP = EA * FB;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int col[NP];
    double t[NP];
    const unsigned first = spr_products<EA, FB>(i, arp, aci, av, brp, bci, bv, col, t);
    int *ok = tcol + off[i];
    double *ov = tval + off[i];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (!((first >> p) & 1u)) continue;
        int r;
        const double s = spr_sum<NP>(p, first, col, t, r);
        ok[r] = col[p];
        ov[r] = s;
    }
    cnt[i] = __popc(first);
}

// The same on C's known pattern (refreshed and learned Galerkin products):
// the row's distinct columns must be exactly C's row, else flag bit 256.
template <int EA, int FB>
__global__ void __launch_bounds__(256) k_spgemm_reg_numeric(int m, const int *__restrict__ arp,
                                                            const int *__restrict__ aci, const double *__restrict__ av,
                                                            const int *__restrict__ brp, const int *__restrict__ bci,
                                                            const double *__restrict__ bv, const int *__restrict__ crp,
                                                            const int *__restrict__ cci, double *__restrict__ cv,
                                                            int *flag) {
    constexpr int NP = EA * FB;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int col[NP];
    double t[NP];
    const unsigned first = spr_products<EA, FB>(i, arp, aci, av, brp, bci, bv, col, t);
    const int c0 = crp[i], len = crp[i + 1] - c0;
    bool bad = __popc(first) != len;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (!((first >> p) & 1u)) continue;
        int r;
        const double s = spr_sum<NP>(p, first, col, t, r);
        if (r < len && cci[c0 + r] == col[p])
            cv[c0 + r] = s;
        else
            bad = true;
    }
    if (bad) atomicOr(flag, 256);
}

// G lanes per output row, for rows of up to CAP products: the products are
// expanded into LDS in A's row order (position p), sorted by the key
// (column, p) with a bitonic network, and each distinct column is summed over
// its terms in p order starting from the first term -- the same sum, bit for
// bit, as the sequential accumulation.  Longer rows: lane 0 of the group with
// the global-memory hash.  One wavefront per block; the sort length is the
// wavefront's largest row rounded up to a power of two.
template <int G, int CAP, int SA_CHUNK, typename KEY>
__global__ void __launch_bounds__(64) k_spgemm_sort(int m, const int *__restrict__ arp, const int *__restrict__ aci,
                                                    const double *__restrict__ av, const int *__restrict__ brp,
                                                    const int *__restrict__ bci, const double *__restrict__ bv,
                                                    const int *__restrict__ off, int *__restrict__ tcol,
                                                    double *__restrict__ tval, int *__restrict__ cnt) {
    constexpr int NG = 64 / G;
    constexpr int SA_PER = SA_CHUNK / G;
    static_assert(SA_PER >= 1 && SA_PER <= 2 && SA_PER * G == SA_CHUNK, "chunk of A entries per group");
    // key = column above the position: 32 bits when the columns fit above
    // log2(CAP) position bits, else 64
    constexpr int PB = (sizeof(KEY) == 4) ? (CAP == 256 ? 8 : 10) : 32;
    static_assert(sizeof(KEY) == 8 || (1 << PB) == CAP, "position bits");
    constexpr KEY PMASK = (KEY)(((KEY)1 << PB) - 1);
    __shared__ KEY skey[NG][CAP];
    __shared__ double sval[NG][CAP];
    __shared__ double sa_val[NG][SA_CHUNK];
    __shared__ int sa_beg[NG][SA_CHUNK];
    __shared__ int sa_off[NG][SA_CHUNK + 1];
    const int lane = threadIdx.x, g = lane / G, gl = lane % G;
    const int i = blockIdx.x * NG + g;
    const bool act = i < m;
    int cap = 0, nprod = 0;
    if (act) {
        cap = off[i + 1] - off[i];
        nprod = (cap - 1) / 2;                // the bound kernel stored 2 * products + 1
    }
    const bool big = nprod > CAP;
    const int myP = (act && !big) ? nprod : 0;
    int maxP = myP;
    for (int d = 32; d >= 1; d >>= 1) maxP = max(maxP, __shfl_xor(maxP, d, 64));
    int S = 1;
    while (S < maxP) S <<= 1;
    // expansion, SA_CHUNK entries of A's row at a time: the group loads their
    // columns, values and B-row extents at once, scans the extents, and then
    // every lane fetches its products (product t of the chunk belongs to the
    // entry whose extent holds t), so the loads do not form one serial chain
    const int e0 = (act && !big) ? arp[i] : 0;
    const int ne_row = (act && !big) ? arp[i + 1] - e0 : 0;
    int nchunk = (ne_row + SA_CHUNK - 1) / SA_CHUNK;
    for (int d = 32; d >= 1; d >>= 1) nchunk = max(nchunk, __shfl_xor(nchunk, d, 64));
    int base = 0;
    for (int ch = 0; ch < nchunk; ++ch) {
        const int c0 = ch * SA_CHUNK;
        const int ne = max(0, min(SA_CHUNK, ne_row - c0));
        // entries 2 gl and 2 gl + 1 of the chunk (G = 16 lanes cover 32)
        int len0 = 0, len1 = 0;
        for (int q = gl * SA_PER; q < gl * SA_PER + SA_PER; ++q) {
            int len = 0;
            if (q < ne) {
                const int k = aci[e0 + c0 + q];
                const int f0 = brp[k];
                len = brp[k + 1] - f0;
                sa_val[g][q] = av[e0 + c0 + q];
                sa_beg[g][q] = f0;
            }
            if (q == gl * SA_PER) len0 = len; else len1 += len;
        }
        // exclusive scan of the per-lane sums across the group
        const int mine = len0 + len1;
        int incl = mine;
        for (int d = 1; d < G; d <<= 1) {
            const int y = __shfl_up(incl, d, G);
            if (gl >= d) incl += y;
        }
        const int excl = incl - mine;
        const int total = __shfl(incl, G - 1, G);
        if (gl * SA_PER < SA_CHUNK) {
            sa_off[g][gl * SA_PER] = excl;
            if (SA_PER > 1) sa_off[g][gl * SA_PER + 1] = excl + len0;
        }
        if (gl == 0) sa_off[g][SA_CHUNK] = total;
        __syncthreads();
        for (int t = gl; t < total; t += G) {
            // the last entry q with sa_off[q] <= t (empty extents are skipped)
            int lo = 0, hi = ne - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (sa_off[g][mid] <= t) lo = mid; else hi = mid - 1;
            }
            const int f = sa_beg[g][lo] + (t - sa_off[g][lo]);
            const int p = base + t;
            skey[g][p] = ((KEY)(unsigned)bci[f] << PB) | (KEY)p;
            sval[g][p] = sa_val[g][lo] * bv[f];
        }
        base += total;
        __syncthreads();
    }
    for (int p = myP + gl; p < S; p += G) skey[g][p] = ~(KEY)0;
    __syncthreads();
    // bitonic network; each lane takes compare-exchange pairs (t, t + j)
    for (int k = 2; k <= S; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int u = gl; u < (S >> 1); u += G) {
                const int t = ((u & ~(j - 1)) << 1) | (u & (j - 1));
                const int q = t + j;
                const KEY x = skey[g][t], y = skey[g][q];
                if ((x > y) == ((t & k) == 0)) {
                    skey[g][t] = y;
                    skey[g][q] = x;
                }
            }
            __syncthreads();
        }
    }
    if (!act) return;
    int *ok = tcol + off[i];
    double *ov = tval + off[i];
    if (big) {
        if (gl == 0) spgemm_row(i, arp, aci, av, brp, bci, bv, ok, ov, 1, cap, ok, ov, cnt);
        return;
    }
    const unsigned long long gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (g * G));
    int nh = 0;
    for (int c0 = 0; c0 < myP; c0 += G) {
        const int pos = c0 + gl;
        const bool head = pos < myP && (pos == 0 || (skey[g][pos] >> PB) != (skey[g][pos - 1] >> PB));
        const unsigned long long mask = __ballot(head) & gmask;
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (head) {
            const KEY kh = skey[g][pos];
            const unsigned j = (unsigned)(kh >> PB);
            double acc = sval[g][(unsigned)(kh & PMASK)];
            for (int t = pos + 1; t < myP && (unsigned)(skey[g][t] >> PB) == j; ++t)
                acc = acc + sval[g][(unsigned)(skey[g][t] & PMASK)];
            ok[nh + before] = (int)j;
            ov[nh + before] = acc;
        }
        nh += __popcll(mask);
    }
    if (gl == 0) cnt[i] = nh;
}

void amg_spgemm_compute_sort(int m, int ncols, int maxprod, const int *arp, const int *aci, const double *av,
                             const int *brp, const int *bci, const double *bv, const int *off, int *tcol,
                             double *tval, int *cnt, hipStream_t st) {
    if (m == 0) return;
    const dim3 g4((m + 3) / 4), g1(m), w(64);
    if (maxprod <= 256) {
        if (ncols < (1 << 24))
            hipLaunchKernelGGL((k_spgemm_sort<16, 256, 32, unsigned>), g4, w, 0, st, m, arp, aci, av, brp, bci, bv,
                               off, tcol, tval, cnt);
        else
            hipLaunchKernelGGL((k_spgemm_sort<16, 256, 32, unsigned long long>), g4, w, 0, st, m, arp, aci, av, brp,
                               bci, bv, off, tcol, tval, cnt);
    } else {
        if (ncols < (1 << 22))
            hipLaunchKernelGGL((k_spgemm_sort<64, 1024, 64, unsigned>), g1, w, 0, st, m, arp, aci, av, brp, bci, bv,
                               off, tcol, tval, cnt);
        else
            hipLaunchKernelGGL((k_spgemm_sort<64, 1024, 64, unsigned long long>), g1, w, 0, st, m, arp, aci, av, brp,
                               bci, bv, off, tcol, tval, cnt);
    }
    CPTR_CHECK_LAUNCH();
}

void amg_spgemm_compute(int m, const int *arp, const int *aci, const double *av, const int *brp, const int *bci,
                        const double *bv, const int *off, int *tcol, double *tval, int *cnt, hipStream_t st,
                        bool narrow) {
    if (m == 0) return;
    if (narrow)
        hipLaunchKernelGGL((k_spgemm_reg<SPR_EA, SPR_FB>), dim3(blocks_for(m, 256)), dim3(256), 0, st, m, arp, aci,
                           av, brp, bci, bv, off, tcol, tval, cnt);
    else
        hipLaunchKernelGGL(k_spgemm_compute, dim3(blocks_for(m, SPG_T)), dim3(SPG_T), 0, st, m, arp, aci, av, brp,
                           bci, bv, off, tcol, tval, cnt);
    CPTR_CHECK_LAUNCH();
}

// --------------------------------------------------------------------------
// SpGEMM C = A B on a known pattern of C (a refreshed Galerkin product, or
// the learned hierarchy's, whose patterns are the classical one's): one
// thread per row of C takes the products of its row in A's row order --
// entry e of A's row, then B's row aci[e] in order -- finds each product's
// column in C's row by bisection and adds the product to that entry.  Every
// entry therefore sums its terms in the order of the sequential
// accumulation, starting from the first term (0 + t = t), bit for bit the
// values of the symbolic kernels.  Rows of at most SPN_CAP entries keep
// their columns and sums in LDS (interleaved across the block's threads);
// longer rows work on C's own arrays.  A product whose column is not in C's
// row sets flag bit 256 (a pattern that does not belong to these operands).
// --------------------------------------------------------------------------
constexpr int SPN_T = 64;
constexpr int SPN_CAP = 32;

__device__ inline int spn_find(const int *cols, int stride, int len, int j) {
    int lo = 0, hi = len - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid * stride] < j) lo = mid + 1; else hi = mid;
    }
    return (len > 0 && cols[lo * stride] == j) ? lo : -1;
}

__global__ void __launch_bounds__(SPN_T) k_spgemm_numeric(int m, const int *__restrict__ arp,
                                                          const int *__restrict__ aci, const double *__restrict__ av,
                                                          const int *__restrict__ brp, const int *__restrict__ bci,
                                                          const double *__restrict__ bv, const int *__restrict__ crp,
                                                          const int *__restrict__ cci, double *__restrict__ cv,
                                                          int *flag) {
    __shared__ int scol[SPN_CAP * SPN_T];
    __shared__ double sacc[SPN_CAP * SPN_T];
    const int i = blockIdx.x * SPN_T + threadIdx.x;
    if (i >= m) return;
    const int c0 = crp[i], len = crp[i + 1] - c0;
    const bool lds = len <= SPN_CAP;
    const int *cols = lds ? scol + threadIdx.x : cci + c0;
    double *acc = lds ? sacc + threadIdx.x : cv + c0;
    const int stride = lds ? SPN_T : 1;
    for (int q = 0; q < len; ++q) {
        if (lds) scol[q * SPN_T + threadIdx.x] = cci[c0 + q];
        acc[q * stride] = 0.0;
    }
    bool bad = false;
    for (int e = arp[i]; e < arp[i + 1]; ++e) {
        const int k = aci[e];
        const double a = av[e];
        for (int f = brp[k]; f < brp[k + 1]; ++f) {
            const double t = a * bv[f];
            const int q = spn_find(cols, stride, len, bci[f]);
            if (q < 0) { bad = true; continue; }
            acc[q * stride] = acc[q * stride] + t;
        }
    }
    if (lds)
        for (int q = 0; q < len; ++q) cv[c0 + q] = sacc[q * SPN_T + threadIdx.x];
    if (bad) atomicOr(flag, 256);
}

void amg_spgemm_numeric(int m, const int *arp, const int *aci, const double *av, const int *brp, const int *bci,
                        const double *bv, const int *crp, const int *cci, double *cv, int *flag, hipStream_t st,
                        bool narrow) {
    if (m == 0) return;
    if (narrow)
        hipLaunchKernelGGL((k_spgemm_reg_numeric<SPR_EA, SPR_FB>), dim3(blocks_for(m, 256)), dim3(256), 0, st, m, arp,
                           aci, av, brp, bci, bv, crp, cci, cv, flag);
    else
        hipLaunchKernelGGL(k_spgemm_numeric, dim3(blocks_for(m, SPN_T)), dim3(SPN_T), 0, st, m, arp, aci, av, brp,
                           bci, bv, crp, cci, cv, flag);
    CPTR_CHECK_LAUNCH();
}

// --------------------------------------------------------------------------
// smoother diagonal and the coarsest level
// --------------------------------------------------------------------------
// dinv = 1 / a_ii (Jacobi) or 1 / (a_ii + sign(a_ii) sum_{j!=i} |a_ij|) (l1-Jacobi);
// diag = a_ii; flag bit 32 on a zero diagonal
__global__ void k_diag_inv(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ v, int smoother, double *__restrict__ dinv,
                           double *__restrict__ diag, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double aii = 0.0, l1 = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        if (ci[e] == i) aii = v[e];
        else l1 += fabs(v[e]);
    }
    if (diag) diag[i] = aii;
    double d = aii;
    if (smoother == CPTR_SMOOTH_L1JACOBI) d = aii + ((aii < 0.0) ? -l1 : l1);
    if (d == 0.0) { atomicOr(flag, 32); dinv[i] = 0.0; return; }
    dinv[i] = 1.0 / d;
}

// Diagonal block of one unknown in a system level (unknown-based AMG): row
// o + i keeps the entries whose column lies in [o, o + m), in their order,
// with the column shifted by -o.  One thread per row.
__global__ void k_sub_count(int m, int o, const int *__restrict__ rp, const int *__restrict__ ci,
                            int *__restrict__ cnt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int k = 0;
    for (int e = rp[o + i]; e < rp[o + i + 1]; ++e) k += (ci[e] >= o && ci[e] < o + m);
    cnt[i] = k;
}

__global__ void k_sub_fill(int m, int o, const int *__restrict__ rp, const int *__restrict__ ci,
                           const double *__restrict__ v, const int *__restrict__ srp, int *__restrict__ sci,
                           double *__restrict__ sv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int k = srp[i];
    for (int e = rp[o + i]; e < rp[o + i + 1]; ++e) {
        const int c = ci[e];
        if (c >= o && c < o + m) {
            sci[k] = c - o;
            sv[k] = v[e];
            ++k;
        }
    }
}

__global__ void k_offset_copy(int n, const int *__restrict__ in, int add, int *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i] + add;
}

void amg_submatrix_count(int m, int o, const int *rp, const int *ci, int *cnt, hipStream_t st) {
    if (m == 0) return;
    hipLaunchKernelGGL(k_sub_count, dim3((m + 255) / 256), dim3(256), 0, st, m, o, rp, ci, cnt);
    CPTR_CHECK_LAUNCH();
}

void amg_submatrix_fill(int m, int o, const int *rp, const int *ci, const double *v, const int *srp, int *sci,
                        double *sv, hipStream_t st) {
    if (m == 0) return;
    hipLaunchKernelGGL(k_sub_fill, dim3((m + 255) / 256), dim3(256), 0, st, m, o, rp, ci, v, srp, sci, sv);
    CPTR_CHECK_LAUNCH();
}

void amg_offset_copy(int n, const int *in, int add, int *out, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_offset_copy, dim3((n + 255) / 256), dim3(256), 0, st, n, in, add, out);
    CPTR_CHECK_LAUNCH();
}

// Gershgorin bound of the spectrum of D^{-1} A: the largest row ratio
// sum_j |a_ij| / |a_ii| (row sums in entry order), maximised through the bit
// patterns of the non-negative doubles
__global__ void k_gershgorin(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                             const double *__restrict__ v, unsigned long long *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0, d = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        s += fabs(v[e]);
        if (ci[e] == i) d = v[e];
    }
    const double q = s / fabs(d);
    atomicMax(out, (unsigned long long)__double_as_longlong(q));
}

__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x == 0) *p = 0ull;
}

void amg_gershgorin(int n, const int *rp, const int *ci, const double *v, unsigned long long *out, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, out);
    if (n > 0) hipLaunchKernelGGL(k_gershgorin, dim3((n + 255) / 256), dim3(256), 0, st, n, rp, ci, v, out);
    CPTR_CHECK_LAUNCH();
}

void amg_diag_inv2(int n, const int *rp, const int *ci, const double *v, int smoother, double *dinv, double *diag,
                   int *flag, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_diag_inv, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, rp, ci, v, smoother, dinv, diag,
                       flag);
    CPTR_CHECK_LAUNCH();
}

// aug = [A | I], n x 2n row-major
__global__ void k_dense_aug(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                            const double *__restrict__ v, double *__restrict__ aug) {
    int r = blockIdx.x;
    if (r >= n) return;
    for (int c = threadIdx.x; c < 2 * n; c += blockDim.x) aug[(size_t)r * 2 * n + c] = (c == n + r) ? 1.0 : 0.0;
    __syncthreads();
    for (int e = rp[r] + threadIdx.x; e < rp[r + 1]; e += blockDim.x) aug[(size_t)r * 2 * n + ci[e]] = v[e];
}

// Gauss-Jordan elimination with partial pivoting, without row normalisation,
// in panels of GJ_NB columns.  Column k: the pivot p_k is an unused row with
// the largest |aug[r][k]| (the first such row in k_gj_panel; up to 2^-11
// relative in k_gj_panel_lds, which serves coarse levels of at most 1024
// rows); every row r != p_k gets
// aug[r][c] -= f_rk aug[p_k][c] for c > k with f_rk = aug[r][k] / aug[p_k][k].
// The panel kernel (one workgroup) runs these steps on the panel's own
// columns and records the multipliers F[r][k - k0] (0 for r = p_k).  The
// columns right of the panel then take all steps at once: with
// u_k(c) = aug[p_k][c] - sum_{j<k} F[p_k][j] u_j(c) (the pivot rows' values
// as the sequential steps see them), aug[r][c] -= sum_k F[r][k] u_k(c).
constexpr int GJ_NB = 16;
constexpr int GJ_ROWS = 4;
constexpr int GJ_PANEL_THREADS = 1024;
constexpr int GJ_RB = 8;     // rows per thread with loads in flight together (k_gj_panel)

// Panel kernel, one workgroup: the steps of the panel's columns, the
// multipliers into F.  Thread (row group, panel column): every thread of a
// row computes that row's multiplier, the first one stores it.
__global__ void __launch_bounds__(GJ_PANEL_THREADS) k_gj_panel(int n, int k0, int nb, double *aug, int *used,
                                                                int *pivrow, double *F, int *flag) {
    __shared__ double wv[GJ_PANEL_THREADS / 64];
    __shared__ int wi[GJ_PANEL_THREADS / 64];
    __shared__ int sp;
    const size_t ld = 2 * (size_t)n;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cc = tid % GJ_NB, r0 = tid / GJ_NB, rstep = blockDim.x / GJ_NB;
    for (int kk = 0; kk < nb; ++kk) {
        const int k = k0 + kk;
        // pivot: the first unused row with the largest |value| in column k
        // (a thread's rows are taken GJ_RB at a time, their loads issued
        // together: the rows lie 2n doubles apart, one cache line each)
        double best = -1.0;
        int arg = -1;
        for (int rb = tid; rb < n; rb += GJ_RB * blockDim.x) {
            double a[GJ_RB];
            int u[GJ_RB];
#pragma unroll
            for (int q = 0; q < GJ_RB; ++q) {
                const int r = rb + q * blockDim.x;
                u[q] = (r < n) ? used[r] : 1;
                a[q] = (r < n) ? fabs(aug[(size_t)r * ld + k]) : 0.0;
            }
#pragma unroll
            for (int q = 0; q < GJ_RB; ++q)
                if (!u[q] && a[q] > best) { best = a[q]; arg = rb + q * blockDim.x; }
        }
        for (int d = 32; d >= 1; d >>= 1) {
            const double ov = __shfl_xor(best, d, 64);
            const int oi = __shfl_xor(arg, d, 64);
            if (oi >= 0 && (arg < 0 || ov > best || (ov == best && oi < arg))) { best = ov; arg = oi; }
        }
        if (lane == 0) { wv[wave] = best; wi[wave] = arg; }
        __syncthreads();
        if (tid == 0) {
            double b0 = wv[0];
            int a0 = wi[0];
            for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
                if (wi[w] >= 0 && (a0 < 0 || wv[w] > b0 || (wv[w] == b0 && wi[w] < a0))) { b0 = wv[w]; a0 = wi[w]; }
            sp = (a0 >= 0 && b0 != 0.0) ? a0 : -1;
            if (sp < 0) {
                // singular: the remaining pivots of the panel name row 0 (the
                // kernels queued behind this one stay inside the matrix)
                atomicOr(flag, 64);
                for (int q = k; q < k0 + nb; ++q) pivrow[q] = 0;
            } else {
                pivrow[k] = a0;
                used[a0] = 1;
            }
        }
        __syncthreads();
        const int p = sp;
        if (p < 0) return;
        const double piv = aug[(size_t)p * ld + k];
        const int c = k + 1 + cc;
        const bool upd = (c < k0 + nb);
        const double pc = upd ? aug[(size_t)p * ld + c] : 0.0;
        for (int rb = r0; rb < n; rb += GJ_RB * rstep) {
            double a[GJ_RB], x[GJ_RB];
#pragma unroll
            for (int q = 0; q < GJ_RB; ++q) {
                const int r = rb + q * rstep;
                a[q] = (r < n) ? aug[(size_t)r * ld + k] : 0.0;
                x[q] = (upd && r < n) ? aug[(size_t)r * ld + c] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < GJ_RB; ++q) {
                const int r = rb + q * rstep;
                if (r >= n) break;
                const double f = (r == p) ? 0.0 : a[q] / piv;
                if (cc == 0) F[(size_t)r * nb + kk] = f;
                if (upd && r != p) aug[(size_t)r * ld + c] = x[q] - f * pc;
            }
        }
        __syncthreads();
    }
}

// The same panel steps for at most GJ_LDS_ROWS rows, one thread per row with
// the row's panel values and multipliers in registers.  Each step's pivot row
// is the one value set another thread needs: its owner publishes it in LDS.
// The pivot of column k is chosen by a 32-bit key: the top 22 bits of |value|
// (its exponent and 11 mantissa bits) above 10 bits of (1023 - row), so the
// pivot is an unused row whose |value| is within 2^-11 of the column's
// largest (the lower row among equal keys); the keys meet in an LDS atomicMax,
// filled for column k + 1 by the lanes that update it in step k.  Two barriers
// per step: after the pivot row is published, and after the next keys.
// Multipliers use the pivot's reciprocal.
constexpr int GJ_LDS_ROWS = GJ_PANEL_THREADS;

__device__ inline unsigned gj_key(double a, int r) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(fabs(a));
    return ((unsigned)(bits >> 41) << 10) | (unsigned)(1023 - r);
}

__global__ void __launch_bounds__(GJ_PANEL_THREADS) k_gj_panel_lds(int n, int k0, int nb, double *aug, int *used,
                                                                    int *pivrow, double *F, int *flag) {
    // the multipliers and pivots reach global memory at the end (a barrier
    // also waits for pending global stores)
    __shared__ double prow[GJ_NB];
    __shared__ unsigned K[3];
    __shared__ int piv[GJ_NB];
    const size_t ld = 2 * (size_t)n;
    const int r = threadIdx.x, lane = r & 63;
    const bool own = r < n;
    double row[GJ_NB], fr[GJ_NB];
    bool usedr = true;
#pragma unroll
    for (int q = 0; q < GJ_NB; ++q) {
        row[q] = 0.0;
        fr[q] = 0.0;
    }
    if (own) {
        usedr = used[r] != 0;
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q)
            if (q < nb) row[q] = aug[(size_t)r * ld + k0 + q];
    }
    if (r < 3) K[r] = 0u;
    __syncthreads();
    unsigned key = (own && !usedr) ? gj_key(row[0], r) : 0u;
    for (int d = 32; d >= 1; d >>= 1) key = max(key, (unsigned)__shfl_xor((int)key, d, 64));
    if (lane == 0 && key) atomicMax(&K[0], key);
    __syncthreads();
    int done = nb;
    // the steps unrolled: the register arrays are then indexed by constants
    // (go and the step test are uniform over the workgroup, so every thread
    // meets the same barriers)
    bool go = true;
#pragma unroll
    for (int kk = 0; kk < GJ_NB; ++kk) {
        if (go && kk < nb) {
            // K[kk % 3] is complete; K[(kk + 1) % 3] collects the next
            // column's keys; K[(kk + 2) % 3] was read one step ago and is
            // cleared for reuse
            const unsigned kv = K[kk % 3];
            const int p = 1023 - (int)(kv & 1023u);
            if ((kv >> 10) == 0u) {
                done = kk;
                go = false;
            } else {
                if (r == 0) {
                    piv[kk] = p;
                    K[(kk + 2) % 3] = 0u;
                }
                if (r == p) {
#pragma unroll
                    for (int q = kk; q < GJ_NB; ++q)
                        if (q < nb) prow[q] = row[q];
                }
                __syncthreads();   // the pivot row is published
                const double rinv = 1.0 / prow[kk];
                unsigned nkey = 0u;
                if (own) {
                    const double f = (r == p) ? 0.0 : row[kk] * rinv;
                    fr[kk] = f;
                    if (r == p) {
                        usedr = true;
                    } else {
#pragma unroll
                        for (int q = kk + 1; q < GJ_NB; ++q)
                            if (q < nb) row[q] -= f * prow[q];
                    }
                    if (!usedr && kk + 1 < nb) nkey = gj_key(row[kk + 1 < GJ_NB ? kk + 1 : kk], r);
                }
                for (int d = 32; d >= 1; d >>= 1) nkey = max(nkey, (unsigned)__shfl_xor((int)nkey, d, 64));
                if (lane == 0 && nkey) atomicMax(&K[(kk + 1) % 3], nkey);
                __syncthreads();   // every thread has read the pivot row; the next keys are in
            }
        }
    }
    __syncthreads();
    if (done < nb && r == 0) atomicOr(flag, 64);
    // (after a singular column the remaining pivots name row 0, so that the
    // kernels still queued behind this one index inside the matrix; the call
    // reports the singular operator)
    if (r < nb) pivrow[k0 + r] = (r < done) ? piv[r] : 0;
    if (own) {
#pragma unroll
        for (int q = 0; q < GJ_NB; ++q)
            if (q < nb) {
                aug[(size_t)r * ld + k0 + q] = row[q];
                F[(size_t)r * nb + q] = fr[q];
            }
        used[r] = usedr ? 1 : 0;
    }
}

// U[kk][c] = u_k(c) for the columns right of the panel
__global__ void k_gj_pivot_rows(int n, int k0, int nb, const double *__restrict__ aug, const int *__restrict__ pivrow,
                                const double *__restrict__ F, double *__restrict__ U) {
    const size_t ld = 2 * (size_t)n;
    const int c = k0 + nb + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= 2 * n) return;
    double u[GJ_NB];
    for (int kk = 0; kk < nb; ++kk) {
        const int p = pivrow[k0 + kk];
        double v = aug[(size_t)p * ld + c];
        for (int j = 0; j < kk; ++j) v -= F[(size_t)p * nb + j] * u[j];
        u[kk] = v;
        U[(size_t)kk * ld + c] = v;
    }
}

__global__ void k_gj_trailing(int n, int k0, int nb, double *__restrict__ aug, const double *__restrict__ F,
                              const double *__restrict__ U) {
    const size_t ld = 2 * (size_t)n;
    const int c = k0 + nb + blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= 2 * n) return;
    double u[GJ_NB];
    for (int kk = 0; kk < nb; ++kk) u[kk] = U[(size_t)kk * ld + c];
    const int r0 = blockIdx.y * GJ_ROWS, r1 = min(n, r0 + GJ_ROWS);
    for (int r = r0; r < r1; ++r) {
        double a = aug[(size_t)r * ld + c];
        for (int kk = 0; kk < nb; ++kk) a -= F[(size_t)r * nb + kk] * u[kk];
        aug[(size_t)r * ld + c] = a;
    }
}

// inv[k][c] = aug[p_k][n + c] / aug[p_k][k]
__global__ void k_gj_extract(int n, const double *aug, const int *pivrow, double *inv, float *inv32) {
    int k = blockIdx.x;
    if (k >= n) return;
    int p = pivrow[k];
    const size_t ld = 2 * (size_t)n;
    double d = aug[(size_t)p * ld + k];
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        double x = aug[(size_t)p * ld + n + c] / d;
        inv[(size_t)k * n + c] = x;
        if (inv32) inv32[(size_t)k * n + c] = (float)x;
    }
}

void amg_dense_inverse(int n, const int *rp, const int *ci, const double *v, double *aug, int *used, int *pivrow,
                       int *flag, double *inv, float *inv32, double *F, double *U, hipStream_t st) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_dense_aug, dim3(n), dim3(256), 0, st, n, rp, ci, v, aug);
    fill_int(used, 0, n, st);
    const int nby = (n + GJ_ROWS - 1) / GJ_ROWS;
    for (int k0 = 0; k0 < n; k0 += GJ_NB) {
        const int nb = std::min(GJ_NB, n - k0);
        const int width = 2 * n - (k0 + nb);
        const int nbx = (width + 255) / 256;
        if (n <= GJ_LDS_ROWS)
            hipLaunchKernelGGL(k_gj_panel_lds, dim3(1), dim3(GJ_PANEL_THREADS), 0, st, n, k0, nb, aug, used, pivrow,
                               F, flag);
        else
            hipLaunchKernelGGL(k_gj_panel, dim3(1), dim3(GJ_PANEL_THREADS), 0, st, n, k0, nb, aug, used, pivrow, F,
                               flag);
        hipLaunchKernelGGL(k_gj_pivot_rows, dim3(nbx), dim3(256), 0, st, n, k0, nb, aug, pivrow, F, U);
        hipLaunchKernelGGL(k_gj_trailing, dim3(nbx, nby), dim3(256), 0, st, n, k0, nb, aug, F, U);
    }
    hipLaunchKernelGGL(k_gj_extract, dim3(n), dim3(256), 0, st, n, aug, pivrow, inv, inv32);
    CPTR_CHECK_LAUNCH();
}

}  // namespace cptr
