// Last stage of the multi-stage preconditioner: block ILU(0) of the scaled
// matrix (ilu(Abar), Eqs. CPRM1 ff. and CPTR3M3; block variant per the remark
// on cell-wise interleaving) and block Jacobi.
//
// Elimination order: the nx x ny grid is cut into tiles; tiles are coloured
// red/black like a checkerboard; all red tiles come before all black tiles and
// each tile keeps the natural (x fastest) order inside.  ILU(0) in this order
// is a global ILU(0) of Abar.  Red tiles are mutually independent (no 5-point
// coupling between two red tiles), likewise black tiles, so one workgroup per
// tile runs the tile's anti-diagonal wavefront in parallel with all other
// tiles of its colour.  On the 5-point pattern zero fill changes only the
// diagonal blocks:  D_i = Abar_ii - sum_{k lower, (k,i) stored} Abar_ik D_k^{-1} Abar_ki,
// and M = (D + L) D^{-1} (D + U) with L, U the off-diagonal blocks of Abar.
#include "internal.h"

#include <algorithm>

namespace cptr {

constexpr int BL_THREADS = 256;

struct TileGeom {
    int nx, ny, tx, ty, ntx;
};

// cells of tile `tile` at anti-diagonal `lev`: lx in [lo, hi], ly = lev - lx
__device__ inline void tile_dims(const TileGeom &g, int tile, int &x0, int &y0, int &tw, int &th) {
    int tix = tile % g.ntx, tiy = tile / g.ntx;
    x0 = tix * g.tx;
    y0 = tiy * g.ty;
    tw = min(g.tx, g.nx - x0);
    th = min(g.ty, g.ny - y0);
}

template <class T>
__device__ inline T shfl(T v, int src) { return __shfl(v, src, 64); }

// ---------------------------------------------------------------------------
// factorisation: lanes of a group own the rows of one cell's block
// ---------------------------------------------------------------------------
template <int B>
__global__ void __launch_bounds__(BL_THREADS) k_bilu_factor(TileGeom g, const int *__restrict__ tiles,
                                                             const int *__restrict__ color,
                                                             const int *__restrict__ rp, const int *__restrict__ ci,
                                                             const int *__restrict__ tpos,
                                                             const double *__restrict__ abar,
                                                             double *__restrict__ dinv, int *flag,
                                                             int diag_only) {
    constexpr int GPW = 64 / B;               // cell groups per wavefront
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane / B, r = lane % B;
    const bool active_lane = grp < GPW;
    const int slot = wave * GPW + grp;        // cell slot inside the block
    const int slots = (int)(blockDim.x / 64) * GPW;
    const int gbase = grp * B;
    int x0, y0, tw, th;
    tile_dims(g, tiles ? tiles[blockIdx.x] : (int)blockIdx.x, x0, y0, tw, th);
    const int nlev = tw + th - 1;
    for (int lev = 0; lev < nlev; ++lev) {
        const int lo = max(0, lev - th + 1), hi = min(lev, tw - 1);
        for (int base = lo; base <= hi; base += slots) {
            const int lx = base + slot;
            const bool act = active_lane && lx <= hi;
            const int i = act ? (x0 + lx) + g.nx * (y0 + (lev - lx)) : 0;
            double row[B], inv[B];
            int myk = -1;
            bool bad = false;
            if (act) {
                int d = -1;
                for (int e = rp[i]; e < rp[i + 1]; ++e) if (ci[e] == i) d = e;
                for (int c = 0; c < B; ++c) row[c] = abar[(size_t)d * B * B + r * B + c];
                if (!diag_only) {
                    const int ci_ = color[i];
                    for (int e = rp[i]; e < rp[i + 1]; ++e) {
                        const int k = ci[e];
                        if (k == i) continue;
                        const int ck = color[k];
                        if (!(ck < ci_ || (ck == ci_ && k < i))) continue;
                        const int et = tpos[e];               // block (k, i)
                        const double *Aik = abar + (size_t)e * B * B + r * B;
                        const double *Dk = dinv + (size_t)k * B * B;
                        const double *Aki = abar + (size_t)et * B * B;
                        double y[B];
                        for (int c = 0; c < B; ++c) {
                            double t = 0.0;
                            for (int m = 0; m < B; ++m) t += Aik[m] * Dk[m * B + c];
                            y[c] = t;
                        }
                        for (int c = 0; c < B; ++c) {
                            double t = 0.0;
                            for (int m = 0; m < B; ++m) t += y[m] * Aki[m * B + c];
                            row[c] -= t;
                        }
                    }
                }
                for (int c = 0; c < B; ++c) inv[c] = (c == r) ? 1.0 : 0.0;
            }
            // Gauss-Jordan with partial pivoting across the B lanes of the group
            bool used = false;
            for (int k = 0; k < B; ++k) {
                const double mine = (act && !used) ? fabs(row[k]) : -1.0;
                double cand = -2.0;
                int who = 0;
                for (int q = 0; q < B; ++q) {     // first lane with the largest |pivot|
                    const double oc = shfl(mine, gbase + q);
                    if (oc > cand) { cand = oc; who = q; }
                }
                const int p = who;
                if (act && cand <= 0.0) bad = true;
                double prow[B], pinv[B];
                for (int c = 0; c < B; ++c) {
                    prow[c] = shfl(row[c], gbase + p);
                    pinv[c] = shfl(inv[c], gbase + p);
                }
                if (act) {
                    if (r == p) {
                        used = true;
                        myk = k;
                    } else if (!bad) {
                        const double f = row[k] / prow[k];
                        for (int c = 0; c < B; ++c) {
                            row[c] -= f * prow[c];
                            inv[c] -= f * pinv[c];
                        }
                    }
                }
            }
            if (act) {
                if (bad) {
                    atomicMin(flag, i);
                } else {
                    const double dk = row[myk];
                    for (int c = 0; c < B; ++c) dinv[(size_t)i * B * B + myk * B + c] = inv[c] / dk;
                }
            }
            __syncthreads();   // the next level reads this level's D^{-1}
        }
    }
}

void bilu_factor_tiles(const TileSched &ts, int n, int b, const int *rp, const int *ci, const int *tpos,
                       const double *abar, double *dinv, int *flag, int color, int diag_only, hipStream_t st) {
    (void)n;
    const int nt = ts.ntiles[color];
    if (nt == 0) return;
    TileGeom g{ts.nx, ts.ny, ts.tx, ts.ty, ts.ntx};
    // one wavefront per tile when a tile's anti-diagonals fit in it
    const int threads = (std::min(ts.tx, ts.ty) <= 64 / b) ? 64 : BL_THREADS;
#define CASE(BB) case BB: hipLaunchKernelGGL(k_bilu_factor<BB>, dim3(nt), dim3(threads), 0, st, g, ts.tiles[color].p, ts.color.p, rp, ci, tpos, abar, dinv, flag, diag_only); break;
    switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

// ---------------------------------------------------------------------------
// apply: u computed on the fly (Algorithm 2's residual updates), then the
// triangular sweeps.  Modes: 0 forward, 1 forward then backward (the last
// colour), 2 backward.  tw holds t after the forward sweep, w after the
// backward one.  y = w + xT e_T + vP e_P.
// ---------------------------------------------------------------------------
template <class T, int B>
__device__ inline T u_entry(int i, int r, const int *rp, const int *ci, const T *slabT, const T *slabP,
                            const double *rv, const T *xT, const T *vP) {
    T u = (T)rv[(size_t)i * B + r];
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        if (xT) u -= slabT[(size_t)e * B + r] * xT[j];
        if (vP) u -= slabP[(size_t)e * B + r] * vP[j];
    }
    return u;
}

template <class T, int B>
__global__ void __launch_bounds__(BL_THREADS) k_bilu_apply(TileGeom g, int mode, const int *__restrict__ tiles,
                                                            const int *__restrict__ color,
                                                            const int *__restrict__ rp, const int *__restrict__ ci,
                                                            const T *__restrict__ abar, const T *__restrict__ dinv,
                                                            const T *__restrict__ slabT, const T *__restrict__ slabP,
                                                            int ip, int it, const double *__restrict__ rv,
                                                            const T *__restrict__ xT, const T *__restrict__ vP,
                                                            T *__restrict__ tw, double *__restrict__ y) {
    constexpr int GPW = 64 / B;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane / B, r = lane % B;
    const bool active_lane = grp < GPW;
    const int slot = wave * GPW + grp;
    const int slots = (BL_THREADS / 64) * GPW;
    const int gbase = grp * B;
    int x0, y0, twd, th;
    tile_dims(g, tiles[blockIdx.x], x0, y0, twd, th);
    const int nlev = twd + th - 1;
    if (mode == 0 || mode == 1) {
        for (int lev = 0; lev < nlev; ++lev) {
            const int lo = max(0, lev - th + 1), hi = min(lev, twd - 1);
            for (int base = lo; base <= hi; base += slots) {
                const int lx = base + slot;
                const bool act = active_lane && lx <= hi;
                const int i = act ? (x0 + lx) + g.nx * (y0 + (lev - lx)) : 0;
                T s = 0;
                if (act) {
                    s = u_entry<T, B>(i, r, rp, ci, slabT, slabP, rv, xT, vP);
                    const int ci_ = color[i];
                    for (int e = rp[i]; e < rp[i + 1]; ++e) {
                        const int k = ci[e];
                        if (k == i) continue;
                        const int ck = color[k];
                        if (!(ck < ci_ || (ck == ci_ && k < i))) continue;
                        const T *Aik = abar + (size_t)e * B * B + r * B;
                        const T *tk = tw + (size_t)k * B;
                        for (int m = 0; m < B; ++m) s -= Aik[m] * tk[m];
                    }
                }
                T tval = 0;
                const T *Di = dinv + (size_t)i * B * B + r * B;
                for (int c = 0; c < B; ++c) {
                    T sc = shfl(s, gbase + c);
                    if (act) tval += Di[c] * sc;
                }
                if (act) tw[(size_t)i * B + r] = tval;
            }
            __syncthreads();
        }
    }
    if (mode == 1 || mode == 2) {
        for (int lev = nlev - 1; lev >= 0; --lev) {
            const int lo = max(0, lev - th + 1), hi = min(lev, twd - 1);
            for (int base = lo; base <= hi; base += slots) {
                const int lx = base + slot;
                const bool act = active_lane && lx <= hi;
                const int i = act ? (x0 + lx) + g.nx * (y0 + (lev - lx)) : 0;
                T q = 0;
                if (act) {
                    const int ci_ = color[i];
                    for (int e = rp[i]; e < rp[i + 1]; ++e) {
                        const int j = ci[e];
                        if (j == i) continue;
                        const int cj = color[j];
                        if (!(cj > ci_ || (cj == ci_ && j > i))) continue;
                        const T *Aij = abar + (size_t)e * B * B + r * B;
                        const T *wj = tw + (size_t)j * B;
                        for (int m = 0; m < B; ++m) q += Aij[m] * wj[m];
                    }
                }
                T corr = 0;
                const T *Di = dinv + (size_t)i * B * B + r * B;
                for (int c = 0; c < B; ++c) {
                    T qc = shfl(q, gbase + c);
                    if (act) corr += Di[c] * qc;
                }
                if (act) {
                    const T w = tw[(size_t)i * B + r] - corr;
                    tw[(size_t)i * B + r] = w;
                    double yv = (double)w;
                    if (r == it && xT) yv += (double)xT[i];
                    if (r == ip && vP) yv += (double)vP[i];
                    y[(size_t)i * B + r] = yv;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// one-wavefront-per-tile apply (tiles with at most 64/b cells per
// anti-diagonal and at most WT_MAX_CELLS cells).  The tile's wavefront values
// live in LDS; couplings to other tiles (all of another colour, final from an
// earlier launch) are folded in by a parallel pre-pass; the level loop then
// only touches in-tile neighbours, with the next level's matrix rows loaded
// into registers while the current level computes.
// ---------------------------------------------------------------------------
constexpr int WT_MAX_CELLS = 512;   // 64 KB of LDS at b = 8 in FP64

// u = r - Abar[:,T] xT - Abar[:,P] vP, one thread per scalar row (rows of
// the 5-point pattern: at most 5 entries, loaded before the sum)
template <class T, int B>
__global__ void k_stage_residual(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                                 const T *__restrict__ slabT, const T *__restrict__ slabP,
                                 const double *__restrict__ rv, const T *__restrict__ xT, const T *__restrict__ vP,
                                 T *__restrict__ u) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)n * B) return;
    const int i = (int)(t / B), r = (int)(t % B);
    T acc = (T)rv[t];
    const int e0 = rp[i], e1 = rp[i + 1];
    constexpr int ME = 5;
    if (e1 - e0 <= ME) {
        // every operand loaded before the sum, which keeps the row order
        int js[ME];
        T a[ME], x[ME], c[ME], y[ME];
#pragma unroll
        for (int q = 0; q < ME; ++q) js[q] = (e0 + q < e1) ? ci[e0 + q] : 0;
#pragma unroll
        for (int q = 0; q < ME; ++q) {
            const bool on = e0 + q < e1;
            a[q] = (on && xT) ? slabT[(size_t)(e0 + q) * B + r] : (T)0;
            x[q] = (on && xT) ? xT[js[q]] : (T)0;
            c[q] = (on && vP) ? slabP[(size_t)(e0 + q) * B + r] : (T)0;
            y[q] = (on && vP) ? vP[js[q]] : (T)0;
        }
#pragma unroll
        for (int q = 0; q < ME; ++q) {
            if (e0 + q >= e1) break;
            if (xT) acc -= a[q] * x[q];
            if (vP) acc -= c[q] * y[q];
        }
    } else {
        for (int e = e0; e < e1; ++e) {
            const int j = ci[e];
            if (xT) acc -= slabT[(size_t)e * B + r] * xT[j];
            if (vP) acc -= slabP[(size_t)e * B + r] * vP[j];
        }
    }
    u[t] = acc;
}

// Couplings between tiles of different colours, fully parallel (one thread
// per scalar row of the cells on the perimeter of a tile of the target
// colour -- only they have neighbours in other tiles), in place on u:
//   mode 0 (before the black sweep): black rows  u_i -= sum_{red j} Abar_ij t_j
//   mode 1 (before the red backward sweep): red rows  u_i = sum_{black j} Abar_ij w_j
// (the backward sweep takes 0 for the red cells inside a tile)
template <class T, int B>
__global__ void k_cross_tile(int nlist, int mode, const int *__restrict__ cells, const int4 *__restrict__ cross,
                             const int *__restrict__ ci, const T *__restrict__ abar, const T *__restrict__ tw,
                             T *__restrict__ u) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nlist * B) return;
    const int k = (int)(t / B), r = (int)(t % B);
    const int i = cells[k];
    const int4 ent = cross[k];
    const int es[4] = {ent.x, ent.y, ent.z, ent.w};
    const size_t ti = (size_t)i * B + r;
    T acc = (mode == 0) ? u[ti] : (T)0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = es[q];
        if (e < 0) break;
        const int j = ci[e];
        const T *Aij = abar + (size_t)e * B * B + (size_t)r * B;
        const T *vj = tw + (size_t)j * B;
        T d = 0;
#pragma unroll
        for (int m = 0; m < B; ++m) d += Aij[m] * vj[m];
        if (mode == 0) acc -= d; else acc += d;
    }
    u[ti] = acc;
}

// the entries of every listed cell's row that couple it to a tile of the
// other colour, ascending (at most 4 on the 5-point pattern; -1 pads)
__global__ void k_cross_entries(int nlist, const int *__restrict__ cells, const int *__restrict__ color,
                                const int *__restrict__ rp, const int *__restrict__ ci, int4 *__restrict__ cross) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nlist) return;
    const int i = cells[k];
    const int ci_ = color[i];
    int es[4] = {-1, -1, -1, -1};
    int q = 0;
    for (int e = rp[i]; e < rp[i + 1] && q < 4; ++e) {
        const int j = ci[e];
        if (j != i && color[j] != ci_) es[q++] = e;
    }
    cross[k] = make_int4(es[0], es[1], es[2], es[3]);
}

// In-tile neighbour blocks of every cell, gathered once per setup so that the
// level chains below address them arithmetically (no index loads):
// tb[(i*4 + k)*B*B + r*B + c] = Abar_ij[r][c] for j the S (k = 0), W (1),
// E (2), N (3) neighbour of cell i when j lies in i's tile, else 0.
template <class T>
__global__ void k_tile_blocks(int n, int b, int nx, int tx, int ty, const int *__restrict__ rp,
                              const int *__restrict__ ci, const double *__restrict__ abar, T *__restrict__ tb) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int bb = b * b;
    if (t >= (long)n * 4 * bb) return;
    const int el = (int)(t % bb);
    const int k = (int)((t / bb) % 4);
    const int i = (int)(t / (4L * bb));
    const int x = i % nx, y = i / nx;
    const int dx = (k == 1) ? -1 : (k == 2) ? 1 : 0, dy = (k == 0) ? -1 : (k == 3) ? 1 : 0;
    const int xj = x + dx, yj = y + dy;
    T v = 0;
    if (xj >= 0 && xj < nx && yj >= 0 && xj / tx == x / tx && yj / ty == y / ty) {
        const int j = xj + nx * yj;
        for (int e = rp[i]; e < rp[i + 1]; ++e)
            if (ci[e] == j) { v = (T)abar[(size_t)e * bb + el]; break; }
    }
    tb[t] = v;
}

template <class T>
void bilu_tile_blocks(const TileSched &ts, int n, int b, const int *rp, const int *ci, const double *abar, T *tb,
                      hipStream_t st) {
    const long tot = (long)n * 4 * b * b;
    hipLaunchKernelGGL(k_tile_blocks<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, b, ts.nx, ts.tx,
                       ts.ty, rp, ci, abar, tb);
    CPTR_CHECK_LAUNCH();
}
template void bilu_tile_blocks<double>(const TileSched &, int, int, const int *, const int *, const double *,
                                       double *, hipStream_t);
template void bilu_tile_blocks<float>(const TileSched &, int, int, const int *, const int *, const double *,
                                      float *, hipStream_t);

// Level chain of one tile per wavefront.  Every anti-diagonal of a tile has at
// most min(tx, ty) <= 64/B cells, so level `lev` is one step: lane group g owns
// cell lx = lo + g of it.  s0 (forward right-hand side, with the couplings to
// lower-colour tiles already folded in) and q0 (backward: couplings to
// higher-colour tiles) come from u; in-tile neighbour values come from LDS.
// The matrix rows, D^{-1} row and s0/q0/t of the next PF levels are kept in
// flight in a register ring, so the chain waits on memory only when PF levels
// of compute are shorter than one memory latency.
//   mode 0: forward only (t to LDS and global)
//   mode 1: forward then backward (the last colour); w to global, y written
//   mode 2: backward only (t read from global); y written
constexpr int PF = 8;

template <class T, int B>
struct LevelRegs {
    T a0[B], a1[B], d[B];
    T s, tv;
    T add;   // backward: the stage-1/2 correction this lane's row of y takes
};

template <class T, int B>
__global__ void __launch_bounds__(64) k_bilu_wave(TileGeom g, int mode, const int *__restrict__ tiles,
                                                  const T *__restrict__ tb, const T *__restrict__ dinv,
                                                  const T *__restrict__ u, T *__restrict__ tw,
                                                  double *__restrict__ y, int ip, int it, const T *__restrict__ xT,
                                                  const T *__restrict__ vP) {
    constexpr int GPW = 64 / B;
    extern __shared__ unsigned char lds_raw[];
    T *W = reinterpret_cast<T *>(lds_raw);   // t (forward), then w (backward)
    const int lane = threadIdx.x;
    const int grp = lane / B, r = lane % B;
    const bool glane = grp < GPW;
    const int gbase = grp * B;
    const int tile = tiles[blockIdx.x];
    int x0, y0, tw_, th;
    tile_dims(g, tile, x0, y0, tw_, th);
    const int nlev = tw_ + th - 1;
    // this lane group's cell of level lev (false if none)
    auto cell_of = [&](int lev, int &lx, int &ly, int &i) {
        if (!glane || lev < 0 || lev >= nlev) return false;
        const int lo = max(0, lev - th + 1), hi = min(lev, tw_ - 1);
        lx = lo + grp;
        if (lx > hi) return false;
        ly = lev - lx;
        i = (x0 + lx) + g.nx * (y0 + ly);
        return true;
    };
    // loads of level lev into q, issued unconditionally (levels and lane groups
    // without a cell read a clamped, valid cell that is never used) so that the
    // memory counters stay exact across the unrolled ring
    auto load = [&](LevelRegs<T, B> &q, int lev, bool fwd) {
        const int lc = min(max(lev, 0), nlev - 1);
        const int lo = max(0, lc - th + 1), hi = min(lc, tw_ - 1);
        const int lx = min(lo + grp, hi), ly = lc - lx;
        const int i = (x0 + lx) + g.nx * (y0 + ly);
        const T *blk = tb + ((size_t)i * 4 + (fwd ? 0 : 2)) * B * B + r * B;
#pragma unroll
        for (int m = 0; m < B; ++m) q.a0[m] = blk[m];
#pragma unroll
        for (int m = 0; m < B; ++m) q.a1[m] = blk[B * B + m];
        const T *Di = dinv + (size_t)i * B * B + r * B;
#pragma unroll
        for (int c = 0; c < B; ++c) q.d[c] = Di[c];
        q.s = u[(size_t)i * B + r];
        q.tv = tw[(size_t)i * B + r];   // used by the backward-only mode
        // y = w + x_T (T row) + v_P (P row): prefetched with the level, so
        // the chain does not wait for these loads
        q.add = (T)0;
        if (!fwd) {
            if (r == it && xT) q.add = xT[i];
            if (r == ip && vP) q.add = vP[i];
        }
    };
    LevelRegs<T, B> ring[PF];

    if (mode == 0 || mode == 1) {
#pragma unroll
        for (int k = 0; k < PF; ++k) load(ring[k], k, true);
        for (int base = 0; base < nlev; base += PF) {
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int lev = base + k;
                if (lev >= nlev) break;
                int lx = 0, ly = 0, i = 0;
                const bool own = cell_of(lev, lx, ly, i);
                const int loc = lx + tw_ * ly;
                T s = ring[k].s;
                if (own) {
                    // lower in-tile neighbours in ascending order: S, then W
                    if (ly > 0) {
#pragma unroll
                        for (int m = 0; m < B; ++m) s -= ring[k].a0[m] * W[(loc - tw_) * B + m];
                    }
                    if (lx > 0) {
#pragma unroll
                        for (int m = 0; m < B; ++m) s -= ring[k].a1[m] * W[(loc - 1) * B + m];
                    }
                } else {
                    s = 0;
                }
                T tv = 0;
#pragma unroll
                for (int c = 0; c < B; ++c) tv += ring[k].d[c] * shfl(s, gbase + c);
                load(ring[k], lev + PF, true);
                if (own) {
                    W[loc * B + r] = tv;
                    if (mode == 0) tw[(size_t)i * B + r] = tv;
                }
                __syncthreads();
            }
        }
    }
    if (mode == 1 || mode == 2) {
#pragma unroll
        for (int k = 0; k < PF; ++k) load(ring[k], nlev - 1 - k, false);
        for (int base = 0; base < nlev; base += PF) {
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int step = base + k;
                if (step >= nlev) break;
                const int lev = nlev - 1 - step;
                int lx = 0, ly = 0, i = 0;
                const bool own = cell_of(lev, lx, ly, i);
                const int loc = lx + tw_ * ly;
                const bool rim = (lx == 0 || ly == 0 || lx == tw_ - 1 || ly == th - 1);
                T q = (mode == 2 && rim) ? ring[k].s : (T)0;
                T tval = 0;
                if (own) {
                    tval = (mode == 2) ? ring[k].tv : W[loc * B + r];
                    // upper in-tile neighbours in ascending order: E, then N
                    if (lx < tw_ - 1) {
#pragma unroll
                        for (int m = 0; m < B; ++m) q += ring[k].a0[m] * W[(loc + 1) * B + m];
                    }
                    if (ly < th - 1) {
#pragma unroll
                        for (int m = 0; m < B; ++m) q += ring[k].a1[m] * W[(loc + tw_) * B + m];
                    }
                } else {
                    q = 0;
                }
                T corr = 0;
#pragma unroll
                for (int c = 0; c < B; ++c) corr += ring[k].d[c] * shfl(q, gbase + c);
                const T add = ring[k].add;
                load(ring[k], lev - PF, false);
                __syncthreads();   // every lane has read its W entries before they are overwritten
                if (own) {
                    const T w = tval - corr;
                    W[loc * B + r] = w;
                    if (mode == 1) tw[(size_t)i * B + r] = w;
                    double yv = (double)w;
                    if ((r == it && xT) || (r == ip && vP)) yv += (double)add;
                    y[(size_t)i * B + r] = yv;
                }
                __syncthreads();
            }
        }
    }
}

template <class T>
static void bilu_apply_wave(const TileSched &ts, int n, int b, const int *rp, const int *ci, const T *abar,
                            const T *tb, const T *dinv, const T *slabT, const T *slabP, int ip, int it,
                            const double *r, const T *xT, const T *vP, T *u, T *tw, double *y, hipStream_t st) {
    const long nr = (long)n * b;
    const int gr = (int)((nr + 255) / 256);
#define CASE(BB) case BB: hipLaunchKernelGGL((k_stage_residual<T, BB>), dim3(gr), dim3(256), 0, st, n, rp, ci, slabT, slabP, r, xT, vP, u); break;
    switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
    TileGeom g{ts.nx, ts.ny, ts.tx, ts.ty, ts.ntx};
    const size_t lds = (size_t)ts.tx * ts.ty * b * sizeof(T);
    auto launch = [&](int color, int mode) {
        const int nt = ts.ntiles[color];
        if (nt == 0) return;
#define CASE(BB) case BB: hipLaunchKernelGGL((k_bilu_wave<T, BB>), dim3(nt), dim3(64), lds, st, g, mode, ts.tiles[color].p, tb, dinv, u, tw, y, ip, it, xT, vP); break;
        switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
        CPTR_CHECK_LAUNCH();
    };
    if (ts.ntiles[1] == 0) {
        launch(0, 1);
    } else {
        auto cross = [&](int mode) {
            const int color = (mode == 0) ? 1 : 0;
            const long nr_ = (long)ts.nrim[color] * b;
            if (nr_ == 0) return;
            const dim3 grid((unsigned)((nr_ + 255) / 256));
            const int4 *cross = reinterpret_cast<const int4 *>(ts.rim_cross[color].p);
#define CASE(BB) case BB: hipLaunchKernelGGL((k_cross_tile<T, BB>), grid, dim3(256), 0, st, ts.nrim[color], mode, ts.rim[color].p, cross, ci, abar, tw, u); break;
            switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
        };
        launch(0, 0);
        cross(0);
        launch(1, 1);
        cross(1);
        launch(0, 2);
    }
    CPTR_CHECK_LAUNCH();
}

bool bilu_wave_ok(const TileSched &ts, int b) {
    return ts.tx * ts.ty <= WT_MAX_CELLS && std::min(ts.tx, ts.ty) <= 64 / b;
}

template <class T>
void bilu_apply_tiles(const TileSched &ts, int b, const int *rp, const int *ci, const T *abar, const T *tb,
                      const T *dinv, const T *slabT, const T *slabP, int ip, int it, const double *r, const T *xT,
                      const T *vP, T *tw, double *y, hipStream_t st) {
    if (bilu_wave_ok(ts, b) && tb) {
        // tw holds 2 n b values: the stage residual u, then t / w
        const int n = ts.nx * ts.ny;
        bilu_apply_wave<T>(ts, n, b, rp, ci, abar, tb, dinv, slabT, slabP, ip, it, r, xT, vP, tw + (size_t)n * b, tw,
                           y, st);
        return;
    }
    TileGeom g{ts.nx, ts.ny, ts.tx, ts.ty, ts.ntx};
    auto launch = [&](int color, int mode) {
        const int nt = ts.ntiles[color];
        if (nt == 0) return;
#define CASE(BB) case BB: hipLaunchKernelGGL((k_bilu_apply<T, BB>), dim3(nt), dim3(BL_THREADS), 0, st, g, mode, ts.tiles[color].p, ts.color.p, rp, ci, abar, dinv, slabT, slabP, ip, it, r, xT, vP, tw, y); break;
        switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
        CPTR_CHECK_LAUNCH();
    };
    if (ts.ntiles[1] == 0) {
        launch(0, 1);
    } else {
        launch(0, 0);
        launch(1, 1);
        launch(0, 2);
    }
}
template void bilu_apply_tiles<double>(const TileSched &, int, const int *, const int *, const double *,
                                       const double *, const double *, const double *, const double *, int, int,
                                       const double *, const double *, const double *, double *, double *,
                                       hipStream_t);
template void bilu_apply_tiles<float>(const TileSched &, int, const int *, const int *, const float *,
                                      const float *, const float *, const float *, const float *, int, int,
                                      const double *, const float *, const float *, float *, double *, hipStream_t);

// ---------------------------------------------------------------------------
// block Jacobi: y_i = D_i^{-1} u_i + xT e_T + vP e_P   (D_i^{-1} = inv(Abar_ii))
// ---------------------------------------------------------------------------
template <class T, int B>
__global__ void __launch_bounds__(BL_THREADS) k_bj_apply(int n, const int *__restrict__ rp,
                                                          const int *__restrict__ ci, const T *__restrict__ dinv,
                                                          const T *__restrict__ slabT, const T *__restrict__ slabP,
                                                          int ip, int it, const double *__restrict__ rv,
                                                          const T *__restrict__ xT, const T *__restrict__ vP,
                                                          double *__restrict__ y) {
    constexpr int GPW = 64 / B;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = lane / B, r = lane % B;
    const int i = (blockIdx.x * (BL_THREADS / 64) + wave) * GPW + grp;
    const bool act = grp < GPW && i < n;
    const int gbase = grp * B;
    T s = act ? u_entry<T, B>(i, r, rp, ci, slabT, slabP, rv, xT, vP) : (T)0;
    T w = 0;
    const T *Di = dinv + (size_t)(act ? i : 0) * B * B + r * B;
    for (int c = 0; c < B; ++c) {
        T sc = shfl(s, gbase + c);
        if (act) w += Di[c] * sc;
    }
    if (act) {
        double yv = (double)w;
        if (r == it && xT) yv += (double)xT[i];
        if (r == ip && vP) yv += (double)vP[i];
        y[(size_t)i * B + r] = yv;
    }
}

template <class T>
void bj_apply_cells(int n, int b, const int *rp, const int *ci, const T *dinv, const T *slabT, const T *slabP,
                    int ip, int it, const double *r, const T *xT, const T *vP, double *y, hipStream_t st) {
    if (n == 0) return;
    const int cells_per_block = (BL_THREADS / 64) * (64 / b);
    const int nb = (n + cells_per_block - 1) / cells_per_block;
#define CASE(BB) case BB: hipLaunchKernelGGL((k_bj_apply<T, BB>), dim3(nb), dim3(BL_THREADS), 0, st, n, rp, ci, dinv, slabT, slabP, ip, it, r, xT, vP, y); break;
    switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
    CPTR_CHECK_LAUNCH();
}
template void bj_apply_cells<double>(int, int, const int *, const int *, const double *, const double *,
                                     const double *, int, int, const double *, const double *, const double *,
                                     double *, hipStream_t);
template void bj_apply_cells<float>(int, int, const int *, const int *, const float *, const float *,
                                    const float *, int, int, const double *, const float *, const float *,
                                    double *, hipStream_t);

// block Jacobi factors: the same group Gauss-Jordan on every diagonal block
// (the tile kernel with diag_only over a single "tile" per cell is not needed:
// reuse it with a 1 x 1 tile geometry)
void bj_factor_cells(int n, int b, const int *rp, const int *ci, const double *abar, double *dinv, int *flag,
                     const int *all_cells_tiles, hipStream_t st) {
    if (n == 0) return;
    TileGeom g{n, 1, 1, 1, n};
#define CASE(BB) case BB: hipLaunchKernelGGL(k_bilu_factor<BB>, dim3(n), dim3(BL_THREADS), 0, st, g, all_cells_tiles, nullptr, rp, ci, nullptr, abar, dinv, flag, 1); break;
    switch (b) { CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) default: throw Error(CPTR_E_ARG, "block size"); }
#undef CASE
    CPTR_CHECK_LAUNCH();
}

// the BSR pattern must be a subset of the 5-point grid stencil for the tile
// order (flag bit 128 otherwise)
__global__ void k_check_5pt(int n, int nx, const int *__restrict__ rp, const int *__restrict__ ci, int *flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int xi = i % nx, yi = i / nx;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int j = ci[e];
        if (j == i) continue;
        int xj = j % nx, yj = j / nx;
        if (abs(xi - xj) + abs(yi - yj) != 1) { atomicOr(flag, 128); return; }
    }
}

// colour of every cell and the tile lists per colour
__global__ void k_tile_colors(int nx, int ny, int tx, int ty, int *color) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nx * ny) return;
    int x = i % nx, y = i / nx;
    color[i] = ((x / tx) + (y / ty)) & 1;
}

void tiles_build(TileSched &ts, int n, int nx, int ny, int tx, int ty, const int *rp, const int *ci, int *flag,
                 hipStream_t st) {
    ts.nx = nx; ts.ny = ny; ts.tx = tx; ts.ty = ty;
    ts.ntx = (nx + tx - 1) / tx;
    ts.nty = (ny + ty - 1) / ty;
    std::vector<int> lists[2];
    for (int t = 0; t < ts.ntx * ts.nty; ++t) lists[((t % ts.ntx) + (t / ts.ntx)) & 1].push_back(t);
    // cells on the perimeter of their tile, per colour
    std::vector<int> rims[2];
    for (int c = 0; c < 2; ++c)
        for (int t : lists[c]) {
            const int x0 = (t % ts.ntx) * tx, y0 = (t / ts.ntx) * ty;
            const int w = std::min(tx, nx - x0), h = std::min(ty, ny - y0);
            for (int ly = 0; ly < h; ++ly)
                for (int lx = 0; lx < w; ++lx)
                    if (lx == 0 || ly == 0 || lx == w - 1 || ly == h - 1) rims[c].push_back(x0 + lx + nx * (y0 + ly));
        }
    for (int c = 0; c < 2; ++c) {
        ts.ntiles[c] = (int)lists[c].size();
        ts.tiles[c].alloc(lists[c].size() + 1);
        if (!lists[c].empty())
            CPTR_HIP(hipMemcpyAsync(ts.tiles[c].p, lists[c].data(), sizeof(int) * lists[c].size(),
                                    hipMemcpyHostToDevice, st));
        ts.nrim[c] = (int)rims[c].size();
        ts.rim[c].alloc(rims[c].size() + 1);
        if (!rims[c].empty())
            CPTR_HIP(hipMemcpyAsync(ts.rim[c].p, rims[c].data(), sizeof(int) * rims[c].size(), hipMemcpyHostToDevice,
                                    st));
    }
    ts.color.alloc(n);
    hipLaunchKernelGGL(k_tile_colors, dim3((n + 255) / 256), dim3(256), 0, st, nx, ny, tx, ty, ts.color.p);
    hipLaunchKernelGGL(k_check_5pt, dim3((n + 255) / 256), dim3(256), 0, st, n, nx, rp, ci, flag);
    for (int c = 0; c < 2; ++c) {
        ts.rim_cross[c].alloc(4 * ((size_t)ts.nrim[c] + 1));
        if (ts.nrim[c] > 0)
            hipLaunchKernelGGL(k_cross_entries, dim3((ts.nrim[c] + 255) / 256), dim3(256), 0, st, ts.nrim[c],
                               ts.rim[c].p, ts.color.p, rp, ci, reinterpret_cast<int4 *>(ts.rim_cross[c].p));
    }
    CPTR_HIP(hipStreamSynchronize(st));   // host lists must outlive the copies
    CPTR_CHECK_LAUNCH();
}

}  // namespace cptr
