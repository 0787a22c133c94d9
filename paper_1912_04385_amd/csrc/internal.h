// Internal declarations of the MI355X multi-stage GMRES library.
// Host orchestration lives in host.cpp; kernels in k_*.hip; this header holds
// the device-buffer helper, the error type and the kernel launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <memory>
#include <vector>

#include "cptr.h"

namespace cptr {

// ---------------------------------------------------------------------------
// errors: internal code throws, the C ABI converts to a status
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
    cptr_status status;
    Error(cptr_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define CPTR_HIP(x)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess)                                                              \
            throw ::cptr::Error(e_ == hipErrorOutOfMemory ? CPTR_E_OOM : CPTR_E_HIP,        \
                                std::string(#x) + ": " + hipGetErrorString(e_));            \
    } while (0)

#define CPTR_CHECK_LAUNCH() CPTR_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// device memory: a caching pool per (device, stream).  Blocks released by a
// buffer go back to the pool of the stream they were allocated for and are
// reused by later allocations on that stream (stream order makes the reuse
// safe); cptr_destroy returns the idle blocks of its stream to the driver.
// Every API entry point names its stream with StreamScope.
// ---------------------------------------------------------------------------
hipStream_t current_stream();
void *pool_alloc(size_t bytes, size_t *cap, hipStream_t *owner, int *dev);
void pool_free(void *p, size_t cap, hipStream_t owner, int dev);
void pool_trim(hipStream_t s);

struct StreamScope {
    hipStream_t prev;
    explicit StreamScope(hipStream_t s);
    ~StreamScope();
};

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    size_t cap = 0;              // bytes of the pooled block
    hipStream_t owner = nullptr;
    int dev = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n), cap(o.cap), owner(o.owner), dev(o.dev) {
        o.p = nullptr; o.n = 0; o.cap = 0;
    }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; cap = o.cap; owner = o.owner; dev = o.dev;
            o.p = nullptr; o.n = 0; o.cap = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void release() {
        if (p) pool_free(p, cap, owner, dev);
        p = nullptr;
        n = 0;
        cap = 0;
    }
    // (re)allocate to at least m elements; contents undefined
    void alloc(size_t m) {
        if (m <= n && p) return;
        release();
        p = (T *)pool_alloc((m ? m : 1) * sizeof(T), &cap, &owner, &dev);
        n = cap / sizeof(T);
    }
    T *get() const { return p; }
};

// scalar CSR operator on the device
struct CsrD {
    int n = 0, ncols = 0, nnz = 0;
    const int *rp = nullptr, *ci = nullptr;   // may alias storage owned elsewhere
    DBuf<int> rp_own, ci_own;
    DBuf<double> v;
    DBuf<float> v32;
};

struct Level {
    CsrD A;
    // pattern of the product A P formed on the way to the next level's A
    // (kept for refreshing the Galerkin product on new values)
    DBuf<int> ap_rp, ap_ci;
    int ap_nnz = -1;        // -1: not kept
    bool ap_narrow = false; // A P's rows fit the register kernel (A rows <= 5, P rows <= 4)
    DBuf<double> dinv;      // 1 / smoothing diagonal
    DBuf<float> dinv32;
    // five-plane copy of A (vc_ell5_fill) in the preconditioner's precision
    // when this is the fine level of a scalar stage on the 5-point pattern of
    // an ell_nx-wide grid (0: none)
    DBuf<float> ell32;
    DBuf<double> ell64;
    int ell_nx = 0;
    DBuf<int> cf;           // 1 = C, 0 = F (not on the coarsest level)
    double lam_max = 0.0;   // Gershgorin bound of the spectrum of D^{-1} A (Chebyshev smoother)
    CsrD P, R;
    int nc = 0;
    // V-cycle work vectors
    DBuf<double> x, b, r;
    DBuf<float> x32, b32, r32;
    // PMIS / interpolation scratch kept for inspection
    DBuf<unsigned char> strong;
};

// exact block-tridiagonal factors of a grid operator (k_blocktri.hip):
// ng groups of g rows, perm / rowof between operator rows and group-major
// positions, S_y^{-1} (ng x g x g) and G_y = S_y^{-1} U_y ((ng - 1) x g x g)
constexpr int BT_MAX_GROUP = 4096;
struct BlockTri {
    int ng = 0, g = 0;
    DBuf<int> perm, rowof;
    DBuf<double> Sinv, G;
    DBuf<double> z, xw;     // solve work vectors, group-major
};

struct Hierarchy {
    std::vector<Level> L;
    std::unique_ptr<BlockTri> bt;   // exact block-tridiagonal solve of the (single) level
    int ncoarse = 0;
    DBuf<double> cinv;      // dense inverse of the coarsest operator, row-major
    DBuf<unsigned long long> lam_dev;   // per-level Gershgorin bounds (Chebyshev smoother), as bits; grown on demand
    DBuf<float> cinv32;
    bool built = false;
};

// ---------------------------------------------------------------------------
// kernel wrappers (defined in k_*.hip)
// ---------------------------------------------------------------------------
// k_common.hip
void scan_exclusive(const int *in, int *out, int n, int *total_dev, hipStream_t s);   // out[n] = total
// d[0, bytes) to the host buffer hdata_dev (device address of coherent
// pinned memory), then seq to *hseq_dev, after the stream's earlier work
void post_to_host(const void *d, int bytes, void *hdata_dev, unsigned long long *hseq_dev, unsigned long long seq,
                  hipStream_t s);
void gather_ints(const int *a, const int *b, const int *c, int *out, hipStream_t s,
                 const int *d = nullptr);   // out[0..3]; null -> 0
void fill_int(int *p, int v, size_t n, hipStream_t s);
void fill_double(double *p, double v, size_t n, hipStream_t s);
void check_pattern(int n, const int *rp, const int *ci, int *flag_dev, hipStream_t s);
void transpose_index(int n, const int *rp, const int *ci, int *tpos, int *flag_dev, hipStream_t s);
void count_nonfinite(const double *x, size_t n, int *flag_dev, hipStream_t s);
void to_float(const double *x, float *y, size_t n, hipStream_t s);
struct ToFloatJob {
    const double *src;
    float *dst;
    size_t n;
};
constexpr int TF_MAX_JOBS = 32;   // jobs per launch of to_float_multi
void to_float_multi(const ToFloatJob *jobs, int count, hipStream_t s);

// k_decouple.hip
void launch_decouple(int variant, int n, int b, const int *rp, const int *ci, const double *A, int ip, int it,
                     double *abar, double *wp, double *wt, double *beta, int *err, hipStream_t s);
// phase 1 (one thread per cell): weights w_P, w_T, beta and the B_PP / C_TT
// entries (two-stage variant: the elliptic block B_ee, 2n rows [P; T], 4 nnzb
// entries, with ee_v non-null); phase 2 (one wavefront per cell): the scaled
// matrix, slabs, FP32 copies
void launch_decouple_weights(int variant, int n, int b, const int *rp, const int *ci, const double *A, int ip,
                             int it, double *wp, double *wt, double *beta, int *err, double *ctt, double *bpp,
                             int *ee_rp, int *ee_ci, double *ee_v, hipStream_t s);
// Phase 1 for CPTR3 and CPR with the values' non-finite scan folded in
// (nf: bit 16), the B_PP / C_TT entries as launch_decouple_weights gives them
void launch_decouple_weights_rows(int variant, int n, int b, const int *rp, const int *ci, const double *A, int ip,
                                  int it, double *wp, double *wt, double *beta, int *err, int *nf, double *ctt,
                                  double *bpp, hipStream_t s);
void launch_decouple_apply(int variant, int n, int b, const int *rp, const int *ci, const double *A, int ip, int it,
                           const double *wp, const double *wt, const double *beta, double *abar, double *slabT,
                           double *slabP, float *abar32, float *slabT32, float *slabP32, hipStream_t s,
                           int nx = 0, int tx = 0, int ty = 0, float *tb32 = nullptr, double *tb64 = nullptr);
// (tb32 / tb64: also the BILU(0) sweeps' in-tile neighbour blocks of the
// tx x ty tiles of an nx-wide grid, as bilu_tile_blocks gives them)
void launch_scale_rhs(int variant, int n, int b, const double *rhs, int ip, int it, const double *wp,
                      const double *wt, const double *beta, double *out, hipStream_t s);
void launch_unscale(int variant, int n, int b, const double *v, int ip, int it, const double *wp,
                    const double *wt, const double *beta, double *out, hipStream_t s);
void launch_extract(int n, int b, int nnzb, const double *abar, int ip, int it, double *ctt, double *bpp,
                    double *slabT, double *slabP, float *abar32, float *slabT32, float *slabP32, hipStream_t s);

// k_amg_setup.hip
void amg_strength(int n, const int *rp, const int *ci, const double *v, double theta, unsigned char *s,
                  hipStream_t st);
void amg_pmis_init(int n, const int *rp, const int *ci, const unsigned char *s, const int *tpos, uint64_t seed,
                   int *cntT, uint64_t *h, int *state, int *und, hipStream_t st);
void amg_pmis_round(int n, const int *rp, const int *ci, const unsigned char *s, const int *tpos, const int *cntT,
                    const uint64_t *h, int *state, unsigned char *newc, int *und, hipStream_t st);
void amg_exti_bound(int n, const int *rp, const int *ci, const unsigned char *s, const int *cf, int *ub, bool wave,
                    hipStream_t st);
void amg_exti_compute2(int n, const int *rp, const int *ci, const double *v, const unsigned char *s, const int *cf,
                       const int *cidx, const double *dg, int pmax, const int *off, int *tcol, double *tw,
                       double *td, int *cnt, hipStream_t st);
void amg_exti_compute_group(int n, int lanes, const int *rp, const int *ci, const double *v,
                            const unsigned char *s, const int *cf, const int *cidx, const double *dg, int pmax,
                            const int *off, int *tcol, double *tw, double *td, int *cnt, hipStream_t st);
void amg_exti_compute_wave(int n, const int *rp, const int *ci, const double *v, const unsigned char *s,
                           const int *cf, const int *cidx, const double *dg, int pmax, const int *off, int *tcol,
                           double *tw, double *td, int *cnt, hipStream_t st);
void amg_compact(int n, const int *off, const int *tcol, const double *tw, const int *prp, int *pci, double *pv,
                 hipStream_t st);
void amg_transpose(int nr, int nc, int nnz, const int *rp, const int *ci, const double *v, int *rpT, int *ciT,
                   double *vT, int *work, hipStream_t st);
// maxprod (device, may be NULL) receives the largest product count of a row,
// maxprod[1] bit 0 when a row of A, or a row of B it reaches, is too long for
// the register kernel (narrow = false)
void amg_spgemm_bound(int m, const int *arp, const int *aci, const int *brp, int *ub, int *maxprod, hipStream_t st);
void amg_spgemm_compute_sort(int m, int ncols, int maxprod, const int *arp, const int *aci, const double *av,
                             const int *brp, const int *bci, const double *bv, const int *off, int *tcol,
                             double *tval, int *cnt, hipStream_t st);
// C = A B on C's known pattern (crp, cci); flag bit 256: a product outside it
// (narrow: the rows fit the register kernel, and C's pattern is exactly the
// product's)
void amg_spgemm_numeric(int m, const int *arp, const int *aci, const double *av, const int *brp, const int *bci,
                        const double *bv, const int *crp, const int *cci, double *cv, int *flag, hipStream_t st,
                        bool narrow = false);
// narrow: every row within the register kernel's limits (the shape word 0)
void amg_spgemm_compute(int m, const int *arp, const int *aci, const double *av, const int *brp, const int *bci,
                        const double *bv, const int *off, int *tcol, double *tval, int *cnt, hipStream_t st,
                        bool narrow = false);
// rows and columns [o, o + m) of a CSR matrix with sorted rows: entry counts,
// then the entries in their order with columns shifted by -o
void amg_submatrix_count(int m, int o, const int *rp, const int *ci, int *cnt, hipStream_t st);
void amg_submatrix_fill(int m, int o, const int *rp, const int *ci, const double *v, const int *srp, int *sci,
                        double *sv, hipStream_t st);
// out[i] = in[i] + add, i < n
void amg_offset_copy(int n, const int *in, int add, int *out, hipStream_t st);
// *out = the bit pattern of max_i sum_j |a_ij| / |a_ii| (a Gershgorin bound of
// the spectrum of D^{-1} A), for the Chebyshev smoother
void amg_gershgorin(int n, const int *rp, const int *ci, const double *v, unsigned long long *out, hipStream_t st);
void amg_diag_inv2(int n, const int *rp, const int *ci, const double *v, int smoother, double *dinv, double *diag,
                   int *flag, hipStream_t st);
// F: n * 16 doubles, U: 16 * 2n doubles (panel multipliers and pivot rows)
void amg_dense_inverse(int n, const int *rp, const int *ci, const double *v, double *aug, int *used, int *pivrow,
                       int *flag, double *inv, float *inv32, double *F, double *U, hipStream_t st);

// k_vcycle.hip (double and float instantiations)
template <class T>
void vc_presmooth_residual(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T omega,
                           const T *b, T *x, T *r, hipStream_t st);
template <class T>
void vc_spmv(int n, int nnz, const int *rp, const int *ci, const T *v, const T *x, T *y, hipStream_t st);
template <class T>
void vc_sweep_residual(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T omega,
                       const T *b, const T *x, const T *r, T *xout, T *rout, hipStream_t st);
template <class T>
void vc_prolong_add(int n, int nnz, const int *rp, const int *ci, const T *v, const T *xc, T *x, hipStream_t st);
template <class T>
void vc_prolong_to(int n, int nnz, const int *rp, const int *ci, const T *v, const T *xc, const T *xin, T *xout,
                   hipStream_t st);
template <class T>
void vc_smooth(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T omega, const T *b,
               const T *xin, T *xout, hipStream_t st);
// the fine level of a scalar stage on the 5-point pattern of an nx-wide grid
// as five coefficient planes (columns i - nx, i - 1, i, i + 1, i + nx), and
// the Jacobi sweeps on them (same results as the CSR kernels)
template <class T>
void vc_ell5_fill(int n, int nx, const int *rp, const int *ci, const T *v, T *ell, hipStream_t st);
template <class T>
void vc_ell5_presmooth_residual(int n, int nx, const T *ell, const T *dinv, T omega, const T *b, T *x, T *r,
                                hipStream_t st);
template <class T>
void vc_ell5_sweep_residual(int n, int nx, const T *ell, const T *dinv, T omega, const T *b, const T *x, const T *r,
                            T *xout, T *rout, hipStream_t st);
template <class T>
void vc_ell5_smooth(int n, int nx, const T *ell, const T *dinv, T omega, const T *b, const T *xin, T *xout,
                    hipStream_t st);
// flag bit 512 when some entry of the n-row pattern lies outside the 5-point
// stencil of an nx-wide grid (columns i - nx, i - 1, i, i + 1, i + nx)
void check_grid5(int n, int nx, const int *rp, const int *ci, int *flag_dev, hipStream_t s);
template <class T>
void vc_residual(int n, int nnz, const int *rp, const int *ci, const T *v, const T *b, const T *x, T *r,
                 hipStream_t st);
template <class T>
void vc_cheb_init(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, const T *b, const T *x,
                  T *x0, T *r, T *d, T theta, hipStream_t st);
template <class T>
void vc_cheb_step(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, const T *din, T *x, T *r,
                  T *dout, T c1, T c2, hipStream_t st);
template <class T>
void vc_dense_apply(int n, const T *Minv, const T *b, T *x, hipStream_t st);
void vc_dense_apply_mixed(int n, const double *Minv, const float *b, float *x, hipStream_t st);
template <class T>
void ms_stage_input(int n, int b, const int *rp, const int *ci, const T *cpl, int comp, const double *r,
                    const T *xs, T *out, hipStream_t st);
void ms_gather_comp(int nnzb, int b, const double *slab, int comp, double *out, float *out32, hipStream_t st);

void vc_hash_uniform(int n, uint64_t seed, double *e, hipStream_t st);
void vc_sub(int n, const double *x, double *e, hipStream_t st);
void vc_spmv_to_float(int n, const int *rp, const int *ci, const double *v, const double *x, float *y,
                      hipStream_t st);
void vc_sub_float(int n, const float *x, double *e, hipStream_t st);

// k_learned.hip: edge-MLP correction of the fine-level temperature interpolation
constexpr int MLP_NF = 16, MLP_NH = 64;
constexpr int MLP_NPARAMS = MLP_NH * MLP_NF + MLP_NH + MLP_NH * MLP_NH + MLP_NH + MLP_NH + 1;
constexpr int MLP_MAX_BLOCKS = 512;
static_assert(MLP_NPARAMS == CPTR_MLP_NPARAMS, "parameter blob size");
void ln_edge_count(int n, const int *cf, const int *cidx, const int *prp, int *cnt, int *isf, int *fine_of,
                   hipStream_t s);
void ln_edge_rows(int n, const int *isf, const int *fpos, const int *estart_row, int *frows, int *estart,
                  hipStream_t s);
void ln_edge_features(int nf, const int *frows, const int *estart, const int *rp, const int *ci, const double *v,
                      const unsigned char *strong, const int *prp, const int *pci, const double *pv,
                      const int *fine_of, float *X, hipStream_t s);
int ln_mlp_waves(int E);
void ln_mlp_forward(int E, const float *X, const float *params, float *o, hipStream_t s);
void ln_learned_weights(int nf, const int *frows, const int *estart, const int *prp, const double *pv,
                        const float *o, double *pv_out, hipStream_t s);
void ln_interp_loss(int nf, int n, int K, const int *frows, const int *estart, const int *prp, const int *pci,
                    const double *pv, const int *fine_of, const double *Ev, const float *o, double *lossrow,
                    float *dout, hipStream_t s);
void ln_jacobi_zero(int n, const int *rp, const int *ci, const double *v, double omega, const double *ein,
                    double *eout, hipStream_t s);
void ln_mlp_backward(int E, const float *X, const float *params, const float *dout, float *part, hipStream_t s);
void ln_grad_reduce(int nw, const float *part, float *grad, hipStream_t s);
void ln_adam(float *p, float *m, float *v, const float *g, double lr, double b1, double b2, double eps, int t,
             hipStream_t s);

// k_blocktri.hip: exact block-tridiagonal solves of grid operators
void bt_check(int n, const int *rp, const int *ci, const int *perm, int g, int *flag, hipStream_t s);
void bt_dense_index(int g, int *drp, int *dci, hipStream_t s);
void bt_schur(int y, int g, const int *rp, const int *ci, const double *v, const int *perm, const int *rowof,
              const double *Gprev, double *S, hipStream_t s);
void bt_g(int y, int g, const int *atrp, const int *atci, const double *atv, const int *perm, const int *rowof,
          const double *Sinv, double *G, hipStream_t s);
template <class T>
void bt_solve(int ng, int g, const int *rp, const int *ci, const double *v, const int *perm, const int *rowof,
              const double *Sinv, const double *G, double *z, double *xw, const T *b, T *x, hipStream_t s);

// k_condense.hip: static condensation of the full Newton system
void launch_condense_cells(int n, int n1, int n2, const double *J21, const double *J22, const double *r2, double *Q,
                           double *q, int *flag, hipStream_t st);
void launch_condense_blocks(int n, int n1, int n2, const int *rp, const int *ci, const double *J11, const double *J12,
                            const double *Q, const double *q, const double *r1, double *A, double *b,
                            hipStream_t st);
void launch_condense_wells(int nwells, int n1, int nw, const int *rp, const int *ci, const int *wcell,
                           const double *J1w, const double *Jw1, const double *Jww, const double *rw, double *A,
                           double *b, double *Qw, double *qw, int *flag, hipStream_t st);
void launch_recover_wells(int nwells, int n1, int nw, const int *wcell, const double *Qw, const double *qw,
                          const double *d1, double *dw, hipStream_t st);
void launch_condense_recover(int n, int n1, int n2, const double *Q, const double *q, const double *d1, double *d2,
                             hipStream_t st);

// k_bilu.hip: BILU(0) in tile order / block Jacobi
struct TileSched {
    int nx = 0, ny = 0, tx = 0, ty = 0, ntx = 0, nty = 0;
    int ntiles[2] = {0, 0};
    DBuf<int> tiles[2];     // tile ids per colour
    DBuf<int> color;        // per cell
    int nrim[2] = {0, 0};
    DBuf<int> rim[2];       // cells on the perimeter of a tile, per colour
    DBuf<int> rim_cross[2]; // per rim cell: its entries to the other colour (4 slots, -1 pads)
};
void tiles_build(TileSched &ts, int n, int nx, int ny, int tx, int ty, const int *rp, const int *ci, int *flag,
                 hipStream_t st);
void bilu_factor_tiles(const TileSched &ts, int n, int b, const int *rp, const int *ci, const int *tpos,
                       const double *abar, double *dinv, int *flag, int color, int diag_only, hipStream_t st);
void bj_factor_cells(int n, int b, const int *rp, const int *ci, const double *abar, double *dinv, int *flag,
                     const int *all_cells_tiles, hipStream_t st);
// last stage apply, fused with Algorithm 2's residual updates:
//   u = r - Abar[:,T] xT - Abar[:,P] vP  (terms dropped when xT / vP are null)
//   w = ilu(Abar)^{-1} u,  y = w + xT e_T + vP e_P
// tb: the in-tile neighbour blocks gathered by bilu_tile_blocks (NULL: the
// multi-wavefront kernel that reads Abar directly)
template <class T>
void bilu_apply_tiles(const TileSched &ts, int b, const int *rp, const int *ci, const T *abar, const T *tb,
                      const T *dinv, const T *slabT, const T *slabP, int ip, int it, const double *r, const T *xT,
                      const T *vP, T *tw, double *y, hipStream_t st);
bool bilu_wave_ok(const TileSched &ts, int b);
template <class T>
void bilu_tile_blocks(const TileSched &ts, int n, int b, const int *rp, const int *ci, const double *abar, T *tb,
                      hipStream_t st);
template <class T>
void bj_apply_cells(int n, int b, const int *rp, const int *ci, const T *dinv, const T *slabT, const T *slabP,
                    int ip, int it, const double *r, const T *xT, const T *vP, double *y, hipStream_t st);

// k_krylov.hip: outer operator and Arnoldi
// streaming read of n doubles, one partial sum per workgroup into part
// (stream_read_blocks(n) entries)
int stream_read_blocks(size_t n);
void launch_stream_read(size_t n, const double *x, double *part, hipStream_t s);
void launch_bsr_spmv(int n, int b, const int *rp, const int *ci, const double *A, const double *x, double *y,
                     hipStream_t s);
void launch_bsr_residual(int n, int b, const int *rp, const int *ci, const double *A, const double *x,
                         const double *rhs, double *r, hipStream_t s);
int kr_nblk(int N);
void kr_mdot(int N, int k, const double *V, size_t ldv, const double *w, double *partial, int nblk,
             hipStream_t st);
void kr_reduce(const double *partial, int nblk, int k, double *out, hipStream_t st);
void kr_update(int N, int k, const double *V, size_t ldv, const double *h, double *w, double *partial, int nblk,
               hipStream_t st);
void kr_norm2_partial(int N, const double *x, double *partial, int nblk, hipStream_t st);
void kr_arnoldi_finish2(int j, int m, double *H, double *cs, double *sn, double *g, const double *hcol,
                        const double *hcol2, const double *nrm_partial, int nblk, double *scal, double *hostinfo,
                        hipStream_t st);
void kr_cycle_prep(const double *nrm_partial, int nblk, int m, double *g, double *scal, double *hostinfo,
                   hipStream_t st);
void kr_scale(int N, const double *w, const double *scal, double *v, hipStream_t st);
void kr_solve_upper(int k, int m, const double *H, const double *g, double *y, hipStream_t st);
template <class TZ>
void kr_combine(int N, int k, const TZ *Z, size_t ldz, const double *y, double *x, hipStream_t st);

}  // namespace cptr
