// Host orchestration of the MI355X multi-stage preconditioned GMRES solver
// and the C ABI declared in cptr.h.  Everything numerical runs in the
// kernels of k_*.hip on the context's stream; the host sequences launches,
// sizes allocations from a few device->host scalars during setup, and reads
// one small status record per Arnoldi step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <memory>
#include <condition_variable>
#include <mutex>
#include <future>
#include <thread>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "internal.h"

using namespace cptr;

static thread_local std::string g_last_error;

static void set_error(const std::string &m) { g_last_error = m; }

constexpr int MAX_COARSE_DENSE = 8192;
constexpr int PMIS_BATCH = 3;            // PMIS rounds between reads of the undecided count
constexpr int PMIS_BATCH_SMALL = 6;      // ... on levels below PMIS_SMALL_LEVEL rows
constexpr int PMIS_SMALL_LEVEL = 100000;
constexpr int SPGEMM_THREAD_CAP = 48;   // LDS hash capacity of the thread-per-row SpGEMM
constexpr double EXTI_SHORT_ROW = 8.0;     // ext+i: 8 lanes per row up to this average row length,
constexpr double EXTI_HALF_WAVE_ROW = 16.0; // then 32 lanes per row up to this one, then 64

// per-hierarchy setup state: each AMG hierarchy is built on its own stream
// (and host thread) with its own scratch and flag word
struct Builder {
    hipStream_t stream = nullptr;
    cptr_options opt{};
    int n = 0, nnzb = 0;
    struct { const int *p = nullptr; } rp, ci;
    DBuf<int> s_i1, s_i2, s_i3, s_i4, flag;
    DBuf<int> stage;             // device ints gathered for one host read
    DBuf<double> s_d1;
    DBuf<uint64_t> s_u1;
    DBuf<unsigned char> s_c1;
    // unknown-based system AMG: the row counts of the unknowns, in row order
    // (empty for a scalar operator), and a second builder (own stream and
    // scratch) that coarsens the second unknown of a level concurrently
    std::vector<int> parts;
    Builder *aux = nullptr;
    int gx = 0, gy = 0;          // grid shape of the cells (0: none), for the exact block-tridiagonal solves
    int ell_nx = 0;              // > 0: the fine level has the 5-point pattern of an ell_nx-wide grid
    int device = 0;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    Builder() = default;
    Builder(const Builder &) = delete;
    Builder &operator=(const Builder &) = delete;
    ~Builder() {
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
    }
};



struct cptr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    cptr_options opt{};
    // problem
    int n = 0, b = 0, nnzb = 0, ip = 0, it = 1, nx = 0, ny = 0;
    bool ready = false;
    bool ell5 = false;   // the block pattern is the 5-point stencil of the nx x ny grid
    DBuf<int> rp, ci, tpos;
    DBuf<double> abar, wp, wt, beta, slabT, slabP;
    DBuf<float> abar32, slabT32, slabP32;
    // the coupling entry of every block that the second scalar stage's input
    // needs: Abar[P,T] (T stage first) or Abar[T,P] (P stage first)
    DBuf<double> cpl;
    DBuf<float> cpl32;
    // last stage
    bool use_tiles = false;
    TileSched ts;
    DBuf<int> cell_list;
    DBuf<double> dinv;
    DBuf<float> dinv32;
    DBuf<double> tb;        // in-tile neighbour blocks of the BILU(0) level chains
    DBuf<float> tb32;
    // scalar stages: 0 = temperature (C_TT), 1 = pressure (B_PP)
    Hierarchy H[2];
    DBuf<double> ctt, bpp;          // level-0 values of the two scalar operators
    // two-stage CPTR: the elliptic block B_ee (2n rows [P; T]); its system
    // hierarchy takes slot 0 of H
    DBuf<int> ee_rp, ee_ci;
    DBuf<double> ee_v;
    double rho[2] = {-1.0, -1.0};   // V-cycle convergence factors measured by update_values
    int reused = 0;                 // bit k: hierarchy k was kept by the last update_values
    // reuse trials after a rejection: the next skip[k] updates rebuild
    // hierarchy k without a trial; skip doubles with every rejection in a row
    int skip_left[2] = {0, 0}, backoff[2] = {1, 1};
    // learned temperature interpolation: parameters and the judge's measurements
    DBuf<float> mlp;
    bool have_mlp = false;
    int used_learned = 0;
    double rho_cls = -1.0, rho_lrn = -1.0;
    DBuf<double> tw;
    DBuf<float> tw32;
    // Krylov workspace
    int m_alloc = 0;
    DBuf<double> V, Z, w, x, rhsbar, r, part, part2, hcol, hcol2, Hm, cs, sn, g, y, scal, hinfo, tmpv;
    double *hinfo_host = nullptr;
    std::vector<double> history;
    DBuf<int> flag;
    // setup scratch
    DBuf<int> s_i1, s_i2, s_i3, s_i4;
    DBuf<double> s_d1, s_d2;
    DBuf<uint64_t> s_u1;
    DBuf<unsigned char> s_c1;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double last_setup_ms = 0.0;
    // per-step stage timing (options.timing)
    hipEvent_t tev[6] = {};
    // concurrent hierarchy builds
    // side streams: 0 temperature hierarchy, 1 pressure hierarchy, 2 the
    // learned temperature hierarchy built beside the classical one
    hipStream_t side[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_dec = nullptr, ev_side[3] = {nullptr, nullptr, nullptr};
    Builder bld[3];
    // the reuse trial of a hierarchy whose last trial failed runs on its own
    // stream beside the speculative rebuild
    hipStream_t side_trial = nullptr;
    Builder bld_trial;
    double tacc[5] = {};
    int tsteps = 0;
    // host wall-clock phases of the last setup: scaling + extraction,
    // temperature and pressure hierarchies (concurrent), last-stage factor
    double tph[4] = {};

    void mark(int k) {
        if (opt.timing) CPTR_HIP(hipEventRecord(tev[k], stream));
    }

    ~cptr_ctx() {
        for (auto &e : tev)
            if (e) (void)hipEventDestroy(e);
        for (int k = 0; k < 3; ++k) {
            if (side[k]) {
                (void)hipStreamSynchronize(side[k]);
                if (k < 2) H[k].L.clear();
                bld[k].~Builder();
                new (&bld[k]) Builder();
                pool_trim(side[k]);
                (void)hipStreamDestroy(side[k]);
            }
            if (ev_side[k]) (void)hipEventDestroy(ev_side[k]);
        }
        if (side_trial) {
            (void)hipStreamSynchronize(side_trial);
            bld_trial.~Builder();
            new (&bld_trial) Builder();
            pool_trim(side_trial);
            (void)hipStreamDestroy(side_trial);
        }
        if (ev_dec) (void)hipEventDestroy(ev_dec);
        if (hinfo_host) (void)hipHostFree(hinfo_host);
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
    }
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Reads of device scalars go through small pinned host buffers: a copy into
// pinned memory is one direct transfer, where pageable memory takes a staged
// copy.  The buffers are kept for reuse until the process ends.
// Host read slots: coherent pinned memory holding a sequence word and up
// to PIN_DATA bytes, each with its device address (slots are reused, never
// freed, across devices: coherent host memory is visible to every GPU)
struct PinSlot {
    unsigned char *h = nullptr;   // host address: [0, 8) sequence word, [8, 8 + PIN_DATA) data
    unsigned char *d = nullptr;   // the same memory's device address
};
static std::mutex g_pin_mu;
static std::vector<PinSlot> g_pin_free;
static std::atomic<unsigned long long> g_pin_seq{1};
constexpr size_t PIN_DATA = 504;
constexpr auto PIN_SPIN = std::chrono::milliseconds(20);   // then wait on the stream

static PinSlot pin_acquire() {
    {
        std::lock_guard<std::mutex> lk(g_pin_mu);
        if (!g_pin_free.empty()) {
            PinSlot p = g_pin_free.back();
            g_pin_free.pop_back();
            return p;
        }
    }
    PinSlot p;
    void *h = nullptr, *d = nullptr;
    CPTR_HIP(hipHostMalloc(&h, 8 + PIN_DATA, hipHostMallocCoherent));
    const hipError_t e = hipHostGetDevicePointer(&d, h, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(h);
        CPTR_HIP(e);
    }
    p.h = (unsigned char *)h;
    p.d = (unsigned char *)d;
    __atomic_store_n((unsigned long long *)p.h, 0ULL, __ATOMIC_RELEASE);
    return p;
}

static void pin_release(PinSlot p) {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    g_pin_free.push_back(p);
}

// copy `bytes` (<= PIN_DATA) from device memory to host after the stream's
// work.  The device posts the bytes and a fresh sequence number into the
// slot (post_to_host) and the host polls the number, which wakes it within
// microseconds of the stream reaching the read; a read still pending after
// PIN_SPIN waits on the stream instead (long queues, and the errors of
// failed kernels, which the stream then reports).
static void read_bytes(void *dst, const void *d, size_t bytes, hipStream_t s) {
    if (bytes > PIN_DATA) throw Error(CPTR_E_ARG, "host read larger than its slot");
    PinSlot p = pin_acquire();
    struct Release {
        PinSlot p;
        ~Release() { pin_release(p); }
    } rel{p};
    const unsigned long long seq = g_pin_seq.fetch_add(1);
    unsigned long long *hseq = (unsigned long long *)p.h;
    post_to_host(d, (int)bytes, p.d + 8, (unsigned long long *)p.d, seq, s);
    const auto t0 = std::chrono::steady_clock::now();
    unsigned it = 0;
    while (__atomic_load_n(hseq, __ATOMIC_ACQUIRE) != seq) {
        if ((++it & 255u) == 0 && std::chrono::steady_clock::now() - t0 > PIN_SPIN) {
            CPTR_HIP(hipStreamSynchronize(s));
            if (__atomic_load_n(hseq, __ATOMIC_ACQUIRE) != seq)
                throw Error(CPTR_E_HIP, "device-to-host read not delivered");
            break;
        }
        __builtin_ia32_pause();
    }
    std::memcpy(dst, p.h + 8, bytes);
}

template <class T>
static T read_scalar(const T *d, hipStream_t s) {
    T v;
    read_bytes(&v, d, sizeof(T), s);
    return v;
}

static int read_flag_and_clear(cptr_ctx *c) {
    int f = read_scalar(c->flag.p, c->stream);
    fill_int(c->flag.p, 0, 1, c->stream);
    return f;
}

static int read_flag_and_clear(Builder *c) {
    int f = read_scalar(c->flag.p, c->stream);
    fill_int(c->flag.p, 0, 1, c->stream);
    return f;
}

static int scan_total(const int *in, int *out, int n, hipStream_t s) {
    scan_exclusive(in, out, n, nullptr, s);
    return read_scalar(out + n, s);
}

// three device ints with one host round trip
static void read_ints3(Builder *c, const int *a, const int *b, const int *d, int out[3]) {
    c->stage.alloc(4);
    gather_ints(a, b, d, c->stage.p, c->stream);
    read_bytes(out, c->stage.p, 3 * sizeof(int), c->stream);
}

// four device ints with one host round trip
static void read_ints4(Builder *c, const int *a, const int *b, const int *d, const int *e, int out[4]) {
    c->stage.alloc(4);
    gather_ints(a, b, d, c->stage.p, c->stream, e);
    read_bytes(out, c->stage.p, 4 * sizeof(int), c->stream);
}

// ---------------------------------------------------------------------------
// AMG hierarchy (setup)
// ---------------------------------------------------------------------------
// SpGEMM C = A B in three phases, so that a caller can batch its host reads:
//   plan:    capacities and their offsets; off[m] = capacity, off[m + 1] =
//            the longest row's product count, off[m + 2] = the shape word
//            (0: every row fits the register kernel) (device)
//   compute: the products into the scratch, row counts, and their scan into
//            C.rp; C.rp[m] = nnz (device)
//   finish:  compaction into C once nnz is known
struct SpgPlan {
    int m = 0;
    DBuf<int> ub, off, cnt;
    DBuf<int> hk;
    DBuf<double> hv;
};

static void spgemm_plan(Builder *c, const CsrD &A, const CsrD &B, SpgPlan &P) {
    hipStream_t s = c->stream;
    const int m = A.n;
    P.m = m;
    P.ub.alloc((size_t)m + 1);
    P.off.alloc((size_t)m + 3);
    P.cnt.alloc((size_t)m + 1);
    amg_spgemm_bound(m, A.rp, A.ci, B.rp, P.ub.p, P.off.p + m + 1, s);
    scan_exclusive(P.ub.p, P.off.p, m, nullptr, s);
}

static void spgemm_compute(Builder *c, const CsrD &A, const CsrD &B, SpgPlan &P, int cap, int maxprod, CsrD &C,
                           int shape = 1) {
    hipStream_t s = c->stream;
    const int m = P.m;
    P.hk.alloc((size_t)cap);
    P.hv.alloc((size_t)cap);
    // rows of at most 5 entries of A times rows of B of at most 4 (shape 0):
    // one thread per row with every product in registers; rows short
    // enough for an LDS hash table: one thread per row; longer rows: lane
    // groups that sort the row's products (all kernels give the same sums,
    // bit for bit)
    const int sk = c->opt.setup_kernels;
    if (sk == 2 || (sk == 0 && 2 * maxprod + 1 <= SPGEMM_THREAD_CAP))
        amg_spgemm_compute(m, A.rp, A.ci, A.v.p, B.rp, B.ci, B.v.p, P.off.p, P.hk.p, P.hv.p, P.cnt.p, s,
                           sk == 0 && shape == 0);
    else
        amg_spgemm_compute_sort(m, B.ncols, maxprod, A.rp, A.ci, A.v.p, B.rp, B.ci, B.v.p, P.off.p, P.hk.p, P.hv.p,
                                P.cnt.p, s);
    C.n = m;
    C.ncols = B.ncols;
    C.rp_own.alloc((size_t)m + 1);
    scan_exclusive(P.cnt.p, C.rp_own.p, m, nullptr, s);
    C.rp = C.rp_own.p;
}

static void spgemm_finish(Builder *c, SpgPlan &P, int nnz, CsrD &C) {
    C.nnz = nnz;
    C.ci_own.alloc((size_t)nnz);
    C.v.alloc((size_t)nnz);
    amg_compact(P.m, P.off.p, P.hk.p, P.hv.p, C.rp_own.p, C.ci_own.p, C.v.p, c->stream);
    C.ci = C.ci_own.p;
    P.hk.release();
    P.hv.release();
}

static void csr_spgemm(Builder *c, const CsrD &A, const CsrD &B, CsrD &C) {
    SpgPlan P;
    spgemm_plan(c, A, B, P);
    int tm[3];
    read_ints3(c, P.off.p + A.n, P.off.p + A.n + 1, P.off.p + A.n + 2, tm);
    spgemm_compute(c, A, B, P, tm[0], tm[1], C, tm[2]);
    spgemm_finish(c, P, read_scalar(C.rp_own.p + A.n, c->stream), C);
}

static void csr_transpose(Builder *c, const CsrD &P, CsrD &R) {
    hipStream_t s = c->stream;
    R.n = P.ncols;
    R.ncols = P.n;
    R.nnz = P.nnz;
    R.rp_own.alloc((size_t)R.n + 1);
    R.ci_own.alloc((size_t)R.nnz);
    R.v.alloc((size_t)R.nnz);
    c->s_i4.alloc((size_t)R.n + 1);
    amg_transpose(P.n, P.ncols, P.nnz, P.rp, P.ci, P.v.p, R.rp_own.p, R.ci_own.p, R.v.p, c->s_i4.p, s);
    R.rp = R.rp_own.p;
    R.ci = R.ci_own.p;
}

static void level_vectors(Level &L, int n, bool fp32) {
    L.x.alloc(n);
    L.b.alloc(n);
    L.r.alloc(3 * (size_t)n);   // r and the ping-pong buffers of the smoother
    if (fp32) {
        L.x32.alloc(n);
        L.b32.alloc(n);
        L.r32.alloc(3 * (size_t)n);
    }
}

// Exact sub-solve of a grid operator by block-tridiagonal LU over grid rows
// (no dense limit): groups of nx rows for a scalar operator, of 2 nx rows
// (both unknowns of a grid row) for the elliptic block of the two-stage
// scheme, whose rows come as [P of every cell; T of every cell].
static void bt_build(Builder *c, Hierarchy &h) {
    hipStream_t s = c->stream;
    Level &L = h.L[0];
    const int n = L.A.n;
    const int gx = c->gx, gy = c->gy;
    if (gx <= 0 || gy <= 0)
        throw Error(CPTR_E_ARG, "exact sub-solves of an operator with " + std::to_string(n) +
                                    " rows (above the dense limit of " + std::to_string(MAX_COARSE_DENSE) +
                                    ") need the grid shape (nx, ny)");
    const bool sys = c->parts.size() > 1;
    const int g = sys ? 2 * gx : gx, ng = gy;
    if ((long)g * ng != n) throw Error(CPTR_E_ARG, "operator rows do not match the grid shape");
    if (g > BT_MAX_GROUP)
        throw Error(CPTR_E_ARG, "exact block-tridiagonal sub-solve: a grid row holds " + std::to_string(g) +
                                    " unknowns (at most " + std::to_string(BT_MAX_GROUP) + ")");
    std::vector<int> perm(n), rowof(n);
    for (int r = 0; r < n; ++r) {
        const int u = sys ? r / (gx * gy) : 0, i = sys ? r % (gx * gy) : r;
        const int q = (i / gx) * g + u * gx + i % gx;
        perm[r] = q;
        rowof[q] = r;
    }
    auto bt = std::make_unique<BlockTri>();
    bt->ng = ng;
    bt->g = g;
    bt->perm.alloc(n);
    bt->rowof.alloc(n);
    CPTR_HIP(hipMemcpyAsync(bt->perm.p, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    CPTR_HIP(hipMemcpyAsync(bt->rowof.p, rowof.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    bt_check(n, L.A.rp, L.A.ci, bt->perm.p, g, c->flag.p, s);
    if (read_flag_and_clear(c) & 1)
        throw Error(CPTR_E_ARG, "exact block-tridiagonal sub-solve: the operator couples grid rows more than one apart");
    CsrD AT;
    csr_transpose(c, L.A, AT);
    const size_t gg = (size_t)g * g;
    bt->Sinv.alloc((size_t)ng * gg);
    if (ng > 1) bt->G.alloc((size_t)(ng - 1) * gg);
    bt->z.alloc(n);
    bt->xw.alloc(n);
    DBuf<int> drp, dci, used, piv;
    DBuf<double> S, aug, F, U;
    drp.alloc((size_t)g + 1);
    dci.alloc(gg);
    bt_dense_index(g, drp.p, dci.p, s);
    S.alloc(gg);
    aug.alloc(2 * gg);
    used.alloc(g);
    piv.alloc(g);
    F.alloc((size_t)g * 16);
    U.alloc((size_t)16 * 2 * g);
    for (int y = 0; y < ng; ++y) {
        bt_schur(y, g, L.A.rp, L.A.ci, L.A.v.p, bt->perm.p, bt->rowof.p, y > 0 ? bt->G.p + (y - 1) * gg : nullptr,
                 S.p, s);
        amg_dense_inverse(g, drp.p, dci.p, S.p, aug.p, used.p, piv.p, c->flag.p, bt->Sinv.p + y * gg, nullptr, F.p,
                          U.p, s);
        if (y + 1 < ng)
            bt_g(y, g, AT.rp, AT.ci, AT.v.p, bt->perm.p, bt->rowof.p, bt->Sinv.p + y * gg, bt->G.p + y * gg, s);
    }
    const int f = read_flag_and_clear(c);
    if (f & 64) throw Error(CPTR_E_SINGULAR_BLOCK, "singular block in the exact block-tridiagonal factorisation");
    h.ncoarse = n;
    h.bt = std::move(bt);
}

// coarsest level: dense inverse (FP64, plus an FP32 copy for the precision split)
static void coarse_inverse(Builder *c, Hierarchy &h) {
    hipStream_t s = c->stream;
    const bool fp32 = (c->opt.precond_precision == CPTR_FP32);
    Level &Lc = h.L.back();
    const int nc = Lc.A.n;
    h.bt.reset();
    // exact sub-solves: the dense inverse up to the dense limit, the
    // block-tridiagonal factorisation above it (always with exact_subsolves 2)
    if (c->opt.exact_subsolves == 2 || (c->opt.exact_subsolves == 1 && nc > MAX_COARSE_DENSE)) {
        bt_build(c, h);
        return;
    }
    if (nc > MAX_COARSE_DENSE && c->opt.exact_subsolves)
        throw Error(CPTR_E_ARG, "exact sub-solve of an operator with " + std::to_string(nc) + " rows (the dense limit is " +
                                    std::to_string(MAX_COARSE_DENSE) + ")");
    if (nc > MAX_COARSE_DENSE)
        throw Error(CPTR_E_ARG, "coarsest AMG level has " + std::to_string(nc) +
                                    " rows (more than the dense limit); raise amg_max_levels or lower amg_max_coarse");
    h.ncoarse = nc;
    h.cinv.alloc((size_t)nc * nc);
    if (fp32) h.cinv32.alloc((size_t)nc * nc);
    DBuf<double> aug, F, U;
    DBuf<int> used, piv;
    aug.alloc((size_t)nc * 2 * nc);
    used.alloc(nc);
    piv.alloc(nc);
    F.alloc((size_t)nc * 16);
    U.alloc((size_t)16 * 2 * nc);
    amg_dense_inverse(nc, Lc.A.rp, Lc.A.ci, Lc.A.v.p, aug.p, used.p, piv.p, c->flag.p, h.cinv.p,
                      fp32 ? h.cinv32.p : nullptr, F.p, U.p, s);
    int f = read_flag_and_clear(c);
    if (f & 256) throw Error(CPTR_E_STATE, "Galerkin product outside its kept pattern");
    if (f & 64) throw Error(CPTR_E_SINGULAR_BLOCK, "singular coarsest AMG operator");
    if (f & 32) throw Error(CPTR_E_SINGULAR_BLOCK, "zero diagonal in an AMG level");
}

// FP32 copies of every level's operator, smoother diagonal and transfer operators
// the fine level's five-plane copy for the sweeps in the preconditioner's
// precision (a scalar stage on the 5-point grid pattern: one row per cell)
static void fine_planes(Builder *c, Hierarchy &h) {
    if (c->ell_nx <= 0 || h.L.empty() || h.L[0].A.n != c->n || c->n % c->ell_nx != 0) return;
    Level &L0 = h.L[0];
    if (c->opt.precond_precision == CPTR_FP32) {
        L0.ell32.alloc((size_t)5 * L0.A.n);
        vc_ell5_fill<float>(L0.A.n, c->ell_nx, L0.A.rp, L0.A.ci, L0.A.v32.p, L0.ell32.p, c->stream);
    } else {
        L0.ell64.alloc((size_t)5 * L0.A.n);
        vc_ell5_fill<double>(L0.A.n, c->ell_nx, L0.A.rp, L0.A.ci, L0.A.v.p, L0.ell64.p, c->stream);
    }
    L0.ell_nx = c->ell_nx;
}

static void hierarchy_fp32(Builder *c, Hierarchy &h) {
    if (c->opt.precond_precision != CPTR_FP32) {
        fine_planes(c, h);
        return;
    }
    std::vector<ToFloatJob> jobs;
    for (auto &L : h.L) {
        L.A.v32.alloc((size_t)L.A.nnz + 1);
        jobs.push_back({L.A.v.p, L.A.v32.p, (size_t)L.A.nnz});
        L.dinv32.alloc(L.A.n);
        jobs.push_back({L.dinv.p, L.dinv32.p, (size_t)L.A.n});
        if (L.P.nnz) {
            L.P.v32.alloc(L.P.nnz);
            jobs.push_back({L.P.v.p, L.P.v32.p, (size_t)L.P.nnz});
            L.R.v32.alloc(L.R.nnz);
            jobs.push_back({L.R.v.p, L.R.v32.p, (size_t)L.R.nnz});
        }
    }
    to_float_multi(jobs.data(), (int)jobs.size(), c->stream);
    fine_planes(c, h);
}

// Build the hierarchy of a scalar operator whose level-0 pattern is the BSR
// pattern (rp, ci owned by the context) and whose values are `vals` (copied).
// ---------------------------------------------------------------------------
// learned fine-level interpolation (T stage): edges, features, MLP, weights
// ---------------------------------------------------------------------------
struct EdgeSet {
    int nf = 0, E = 0;
    DBuf<int> frows, estart, fine_of, cidx;
    DBuf<float> X;
};

// the F-row edges of a level's (classical) interpolation and their features
static void edges_build(hipStream_t s, const Level &L, EdgeSet &es) {
    const int n = L.A.n;
    DBuf<int> cnt, isf, erow, fpos;
    cnt.alloc(n + 1);
    isf.alloc(n + 1);
    erow.alloc(n + 1);
    fpos.alloc(n + 1);
    es.cidx.alloc(n + 1);
    es.fine_of.alloc(L.nc + 1);
    scan_exclusive(L.cf.p, es.cidx.p, n, nullptr, s);
    ln_edge_count(n, L.cf.p, es.cidx.p, L.P.rp, cnt.p, isf.p, es.fine_of.p, s);
    scan_exclusive(cnt.p, erow.p, n, nullptr, s);
    scan_exclusive(isf.p, fpos.p, n, nullptr, s);
    es.E = read_scalar(erow.p + n, s);
    es.nf = read_scalar(fpos.p + n, s);
    es.frows.alloc(es.nf + 1);
    es.estart.alloc(es.nf + 1);
    ln_edge_rows(n, isf.p, fpos.p, erow.p, es.frows.p, es.estart.p, s);
    es.X.alloc((size_t)es.E * MLP_NF + 1);
    ln_edge_features(es.nf, es.frows.p, es.estart.p, L.A.rp, L.A.ci, L.A.v.p, L.strong.p, L.P.rp, L.P.ci, L.P.v.p,
                     es.fine_of.p, es.X.p, s);
}

// replace the F-row weights of level L's interpolation by the learned ones
static void apply_learned(hipStream_t s, Level &L, const float *mlp) {
    EdgeSet es;
    edges_build(s, L, es);
    if (es.E == 0) return;
    DBuf<float> o;
    o.alloc(es.E);
    ln_mlp_forward(es.E, es.X.p, mlp, o.p, s);
    ln_learned_weights(es.nf, es.frows.p, es.estart.p, L.P.rp, L.P.v.p, o.p, L.P.v.p, s);
    CPTR_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// classical coarsening and interpolation of one scalar operator
// ---------------------------------------------------------------------------
// the interpolation's entries before compaction
struct InterpScratch {
    DBuf<int> off, tcol;
    DBuf<double> twt;
};

// Strength, PMIS (random measure indexed by row) and extended+i with
// truncation on the scalar operator A with diagonal dg: the C/F split into cf
// (A.n entries), the strength flags into strong (A.nnz + 1 bytes), the
// interpolation's entries into the scratch and P's row pointers into
// P.rp_own (P.rp_own[A.n] = P's nnz, on the device).  Returns the number of C
// points; P is not formed when that is 0 or A.n.  Row kernels of ext+i: lane
// groups sized by the row length with the rows fetched into LDS (default),
// one wavefront per row (1), one thread per row (2), or 8-lane groups on
// every level (3: rows beyond the groups' LDS caps take the per-row
// sequential path); all give the same interpolation bit for bit.
static int interp_rows(Builder *c, const CsrD &A, const double *dg, int *cf, unsigned char *strong, bool check_sym,
                       InterpScratch &is, CsrD &P) {
    hipStream_t s = c->stream;
    const cptr_options &o = c->opt;
    const int m = A.n;
    c->s_i1.alloc((size_t)A.nnz + 1);      // transpose positions
    transpose_index(m, A.rp, A.ci, c->s_i1.p, c->flag.p, s);
    // Galerkin products P^T A P of a structurally symmetric A are symmetric:
    // only the fine level's pattern needs the check
    if (check_sym && (read_flag_and_clear(c) & 8))
        throw Error(CPTR_E_ARG, "AMG level pattern is not structurally symmetric");
    amg_strength(m, A.rp, A.ci, A.v.p, o.amg_theta, strong, s);
    c->s_i2.alloc((size_t)m + 1);          // |S^T|
    c->s_u1.alloc((size_t)m);              // random measure
    c->s_c1.alloc((size_t)m);              // new C flags
    c->s_i3.alloc(4);                      // undecided counter
    fill_int(c->s_i3.p, 0, 1, s);
    amg_pmis_init(m, A.rp, A.ci, strong, c->s_i1.p, o.pmis_seed, c->s_i2.p, c->s_u1.p, cf, c->s_i3.p, s);
    // rounds run in batches between reads of the undecided count (a round on
    // a fully decided level changes nothing); small levels take longer
    // batches: their rounds are cheap, and their coarsening needs more of them
    const int batch = (m >= PMIS_SMALL_LEVEL) ? PMIS_BATCH : PMIS_BATCH_SMALL;
    int und = 1, rounds = 0;
    while (und > 0) {
        for (int q = 0; q < batch; ++q) {
            fill_int(c->s_i3.p, 0, 1, s);
            amg_pmis_round(m, A.rp, A.ci, strong, c->s_i1.p, c->s_i2.p, c->s_u1.p, cf, c->s_c1.p, c->s_i3.p, s);
        }
        und = read_scalar(c->s_i3.p, s);
        rounds += batch;
        if (rounds > 10000) throw Error(CPTR_E_STATE, "PMIS did not terminate");
    }
    // coarse numbering and the ext+i capacity bound, read together
    DBuf<int> cidx, ub, cnt;
    DBuf<double> td;
    cidx.alloc((size_t)m + 1);
    scan_exclusive(cf, cidx.p, m, nullptr, s);
    ub.alloc(m + 1);
    is.off.alloc(m + 1);
    cnt.alloc(m + 1);
    const double avg_row = (double)A.nnz / (double)m;
    const int ek = o.setup_kernels;
    amg_exti_bound(m, A.rp, A.ci, strong, cf, ub.p, ek == 1 || (ek == 0 && avg_row > EXTI_SHORT_ROW), s);
    scan_exclusive(ub.p, is.off.p, m, nullptr, s);
    int rd[3];
    read_ints3(c, cidx.p + m, is.off.p + m, nullptr, rd);
    const int nc = rd[0], cap = rd[1];
    if (nc == 0 || nc == m) return nc;
    is.tcol.alloc(cap);
    is.twt.alloc(cap);
    td.alloc((size_t)A.nnz + 1);
    if (ek == 2)
        amg_exti_compute2(m, A.rp, A.ci, A.v.p, strong, cf, cidx.p, dg, o.amg_pmax, is.off.p, is.tcol.p, is.twt.p,
                          td.p, cnt.p, s);
    else if (ek == 1)
        amg_exti_compute_wave(m, A.rp, A.ci, A.v.p, strong, cf, cidx.p, dg, o.amg_pmax, is.off.p, is.tcol.p,
                              is.twt.p, td.p, cnt.p, s);
    else
        amg_exti_compute_group(m, (ek == 3 || avg_row <= EXTI_SHORT_ROW) ? 8 : avg_row <= EXTI_HALF_WAVE_ROW ? 32 : 64,
                               A.rp, A.ci, A.v.p, strong, cf, cidx.p, dg, o.amg_pmax, is.off.p, is.tcol.p, is.twt.p,
                               td.p, cnt.p, s);
    P.n = m;
    P.ncols = nc;
    P.rp_own.alloc((size_t)m + 1);
    scan_exclusive(cnt.p, P.rp_own.p, m, nullptr, s);
    P.rp = P.rp_own.p;
    return nc;
}

// P's columns and weights once its nnz (P.nnz) is known
static void compact_interp(Builder *c, InterpScratch &is, CsrD &P) {
    P.ci_own.alloc((size_t)P.nnz + 1);
    P.v.alloc((size_t)P.nnz + 1);
    amg_compact(P.n, is.off.p, is.tcol.p, is.twt.p, P.rp_own.p, P.ci_own.p, P.v.p, c->stream);
    P.ci = P.ci_own.p;
}

// ---------------------------------------------------------------------------
// unknown-based system AMG (two-stage CPTR on B_ee)
// ---------------------------------------------------------------------------
// The scalar coarsening of one unknown's diagonal block Au, diagonal dg
// (interp_rows, then P's size read and P compacted): the C/F split into cf
// (Au.n entries) and P; returns the number of C points (P is left empty when
// that is 0 or Au.n).
static int coarsen_block(Builder *c, const CsrD &Au, const double *dg, int *cf, CsrD &P, bool check_sym) {
    DBuf<unsigned char> strong;
    strong.alloc((size_t)Au.nnz + 1);
    InterpScratch is;
    const int nc = interp_rows(c, Au, dg, cf, strong.p, check_sym, is, P);
    if (nc == 0 || nc == Au.n) return nc;
    P.nnz = read_scalar(P.rp_own.p + Au.n, c->stream);
    compact_interp(c, is, P);
    return nc;
}

// One unknown's diagonal block (rows and columns [o, o + mu) of L.A)
// extracted and coarsened; returns its number of C points.
static int coarsen_unknown(Builder *c, const Level &L, int o, int mu, int *cf, const double *dg, CsrD &P,
                           bool check_sym) {
    hipStream_t s = c->stream;
    CsrD Au;
    Au.n = Au.ncols = mu;
    Au.rp_own.alloc((size_t)mu + 1);
    DBuf<int> cnt;
    cnt.alloc((size_t)mu + 1);
    amg_submatrix_count(mu, o, L.A.rp, L.A.ci, cnt.p, s);
    scan_exclusive(cnt.p, Au.rp_own.p, mu, nullptr, s);
    Au.rp = Au.rp_own.p;
    Au.nnz = read_scalar(Au.rp_own.p + mu, s);
    Au.ci_own.alloc((size_t)Au.nnz + 1);
    Au.v.alloc((size_t)Au.nnz + 1);
    amg_submatrix_fill(mu, o, L.A.rp, L.A.ci, L.A.v.p, Au.rp, Au.ci_own.p, Au.v.p, s);
    Au.ci = Au.ci_own.p;
    return coarsen_block(c, Au, dg, cf, P, check_sym);
}

// One level of unknown-based coarsening: the unknowns hold consecutive row
// ranges (parts) of L.  Each unknown's diagonal block is extracted and
// coarsened on its own; P = blockdiag(P_u) (its C points ordered unknown by
// unknown), R = P^T, and the next operator R A P keeps every coupling between
// the unknowns.  Returns false, leaving L the coarsest level, when some
// unknown's block has no C point or no F point; else fills nxt and replaces
// parts by the unknowns' coarse sizes.
static bool coarsen_system(Builder *c, Level &L, std::vector<int> &parts, bool check_sym, Level &nxt) {
    hipStream_t s = c->stream;
    const int m = L.A.n;
    const int nu = (int)parts.size();
    std::vector<CsrD> Ps(nu);
    std::vector<int> ncs(nu), offs(nu, 0);
    for (int u = 1; u < nu; ++u) offs[u] = offs[u - 1] + parts[u - 1];
    DBuf<int> cf;
    cf.alloc((size_t)m + 1);
    Builder *aux = (nu == 2) ? c->aux : nullptr;
    if (aux) {
        // the second unknown on the second builder's stream and host thread:
        // its stream starts after this level's operator and diagonal are
        // ready, and this stream resumes once both blocks are coarsened (its
        // buffers return to its own stream's pool, whose next use is again
        // ordered after this stream)
        if (!c->ev_in) CPTR_HIP(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
        if (!c->ev_out) CPTR_HIP(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
        CPTR_HIP(hipEventRecord(c->ev_in, s));
        std::exception_ptr err;
        std::thread t([&]() {
            try {
                CPTR_HIP(hipSetDevice(aux->device));
                StreamScope scope(aux->stream);
                CPTR_HIP(hipStreamWaitEvent(aux->stream, c->ev_in, 0));
                if (!aux->flag.p) {
                    aux->flag.alloc(4);
                    fill_int(aux->flag.p, 0, 1, aux->stream);
                }
                ncs[1] = coarsen_unknown(aux, L, offs[1], parts[1], cf.p + offs[1], c->s_d1.p + offs[1], Ps[1], false);
                CPTR_HIP(hipEventRecord(c->ev_out, aux->stream));
            } catch (...) {
                err = std::current_exception();
            }
        });
        // on an error, the second stream's queued work (which reads this
        // level) ends before the exception leaves
        try {
            ncs[0] = coarsen_unknown(c, L, 0, parts[0], cf.p, c->s_d1.p, Ps[0], check_sym);
        } catch (...) {
            t.join();
            (void)hipStreamSynchronize(aux->stream);
            throw;
        }
        t.join();
        if (err) {
            (void)hipStreamSynchronize(aux->stream);
            (void)hipStreamSynchronize(s);
            std::rethrow_exception(err);
        }
        CPTR_HIP(hipStreamWaitEvent(s, c->ev_out, 0));
    } else {
        for (int u = 0; u < nu; ++u) {
            ncs[u] = coarsen_unknown(c, L, offs[u], parts[u], cf.p + offs[u], c->s_d1.p + offs[u], Ps[u],
                                     check_sym && u == 0);
            if (ncs[u] == 0 || ncs[u] == parts[u]) return false;
        }
    }
    for (int u = 0; u < nu; ++u)
        if (ncs[u] == 0 || ncs[u] == parts[u]) return false;
    CsrD &P = L.P;
    int nz = 0, nc = 0;
    for (int u = 0; u < nu; ++u) {
        nz += Ps[u].nnz;
        nc += ncs[u];
    }
    P.n = m;
    P.ncols = nc;
    P.nnz = nz;
    P.rp_own.alloc((size_t)m + 1);
    P.ci_own.alloc((size_t)nz + 1);
    P.v.alloc((size_t)nz + 1);
    int ro = 0, co = 0, zo = 0;
    for (int u = 0; u < nu; ++u) {
        // rows u: pointers shifted by the entries before, columns by the
        // coarse points before (the shared boundary pointer is written twice
        // with the same value)
        amg_offset_copy(parts[u] + 1, Ps[u].rp, zo, P.rp_own.p + ro, s);
        amg_offset_copy(Ps[u].nnz, Ps[u].ci, co, P.ci_own.p + zo, s);
        if (Ps[u].nnz)
            CPTR_HIP(hipMemcpyAsync(P.v.p + zo, Ps[u].v.p, sizeof(double) * Ps[u].nnz, hipMemcpyDeviceToDevice, s));
        ro += parts[u];
        co += ncs[u];
        zo += Ps[u].nnz;
    }
    P.rp = P.rp_own.p;
    P.ci = P.ci_own.p;
    L.cf = std::move(cf);
    L.nc = nc;
    csr_transpose(c, P, L.R);
    CsrD AP;
    csr_spgemm(c, L.A, P, AP);
    csr_spgemm(c, L.R, AP, nxt.A);
    parts = ncs;
    return true;
}

// Chebyshev smoother: the Gershgorin bound of level l into the hierarchy's
// device array, and all levels' bounds to the host in one read
static void level_bound(Builder *c, Hierarchy &h, int l) {
    if (c->opt.smoother != CPTR_SMOOTH_CHEBYSHEV) return;
    if (!h.lam_dev.p || (size_t)l >= h.lam_dev.n) {
        // room for 32 levels at first, doubled when a hierarchy goes deeper;
        // the bounds of the levels above are kept
        DBuf<unsigned long long> grown;
        grown.alloc(std::max<size_t>(32, 2 * (size_t)l));
        if (l > 0 && h.lam_dev.p) {
            CPTR_HIP(hipMemcpyAsync(grown.p, h.lam_dev.p, sizeof(unsigned long long) * l, hipMemcpyDeviceToDevice,
                                    c->stream));
            // the old block may belong to another stream's free list
            CPTR_HIP(hipStreamSynchronize(c->stream));
        }
        h.lam_dev = std::move(grown);
    }
    const Level &L = h.L[l];
    amg_gershgorin(L.A.n, L.A.rp, L.A.ci, L.A.v.p, h.lam_dev.p + l, c->stream);
}

static void read_bounds(Builder *c, Hierarchy &h) {
    if (c->opt.smoother != CPTR_SMOOTH_CHEBYSHEV) return;
    std::vector<unsigned long long> bits(h.L.size());
    read_bytes(bits.data(), h.lam_dev.p, sizeof(unsigned long long) * bits.size(), c->stream);
    for (size_t l = 0; l < h.L.size(); ++l) {
        double q;
        std::memcpy(&q, &bits[l], sizeof q);
        h.L[l].lam_max = q;
    }
}

// The levels of a classical build handed to a second build that keeps its
// C/F splits and transfer operators (the learned interpolation's judge).
// The classical builder publishes the fine level once its C/F split and
// classical interpolation are formed (with the fine operator, its smoother
// diagonal and strength flags), and every level once its Galerkin product is
// formed (its interpolation and restriction, and the patterns of A P and of
// the next level's operator, which the second build's products share), each
// with an event recorded on its stream; it closes the feed when it stops
// forming interpolations (or fails).  The published device buffers stay
// unchanged until the classical hierarchy is destroyed, which the caller
// does only after the second build has ended.
struct LevelFeed {
    struct Csr {
        int n = 0, ncols = 0, nnz = 0;
        const int *rp = nullptr, *ci = nullptr;
        const double *v = nullptr;
    };
    struct Item {
        int n = 0, nc = 0;
        const int *cf = nullptr;
        Csr P, R;
        Csr AP, Anext;                              // patterns (values unused)
        bool ap_narrow = false;                     // A P fits the register kernel
        int annz = 0;                               // fine level: the operator
        const double *av = nullptr, *dinv = nullptr;
        const unsigned char *strong = nullptr;
        hipEvent_t ev = nullptr;
    };
    std::mutex mu;
    std::condition_variable cv;
    Item fine;
    bool fine_ready = false;
    std::vector<Item> items;
    bool closed = false;
    LevelFeed() = default;
    LevelFeed(const LevelFeed &) = delete;
    LevelFeed &operator=(const LevelFeed &) = delete;
    ~LevelFeed() {
        if (fine.ev) (void)hipEventDestroy(fine.ev);
        for (auto &it : items)
            if (it.ev) (void)hipEventDestroy(it.ev);
    }
    static Csr view(const CsrD &a) { return {a.n, a.ncols, a.nnz, a.rp, a.ci, a.v.p}; }
    void publish(Item it, hipStream_t s, bool is_fine) {
        CPTR_HIP(hipEventCreateWithFlags(&it.ev, hipEventDisableTiming));
        const hipError_t e = hipEventRecord(it.ev, s);
        {
            std::lock_guard<std::mutex> lk(mu);
            if (is_fine) {
                fine = it;
                fine_ready = true;
            } else {
                items.push_back(it);      // (the destructor releases the events)
            }
        }
        cv.notify_all();
        if (e != hipSuccess) throw Error(CPTR_E_HIP, std::string("hipEventRecord: ") + hipGetErrorString(e));
    }
    void close() {
        {
            std::lock_guard<std::mutex> lk(mu);
            closed = true;
        }
        cv.notify_all();
    }
    // the fine level, or false once the feed closed without it
    bool wait_fine(Item &out) {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return fine_ready || closed; });
        if (!fine_ready) return false;
        out = fine;
        return true;
    }
    // level l's products, or false once the feed closed without them
    bool wait(size_t l, Item &out) {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return items.size() > l || closed; });
        if (items.size() <= l) return false;
        out = items[l];
        return true;
    }
};

static void copy_csr(hipStream_t s, const LevelFeed::Csr &a, CsrD &d, bool values = true) {
    d.n = a.n;
    d.ncols = a.ncols;
    d.nnz = a.nnz;
    d.rp_own.alloc((size_t)a.n + 1);
    d.ci_own.alloc((size_t)a.nnz + 1);
    d.v.alloc((size_t)a.nnz + 1);
    CPTR_HIP(hipMemcpyAsync(d.rp_own.p, a.rp, sizeof(int) * (a.n + 1), hipMemcpyDeviceToDevice, s));
    if (a.nnz) {
        CPTR_HIP(hipMemcpyAsync(d.ci_own.p, a.ci, sizeof(int) * a.nnz, hipMemcpyDeviceToDevice, s));
        if (values) CPTR_HIP(hipMemcpyAsync(d.v.p, a.v, sizeof(double) * a.nnz, hipMemcpyDeviceToDevice, s));
    }
    d.rp = d.rp_own.p;
    d.ci = d.ci_own.p;
}

// the next level's operator A_{l+1} = R (A P) of level L on kept patterns:
// A P (L.ap_*) into scratch, then R (A P) into N.A's values
static void galerkin_numeric(Builder *c, Level &L, Level &N) {
    hipStream_t s = c->stream;
    DBuf<double> apv;
    apv.alloc((size_t)L.ap_nnz + 1);
    amg_spgemm_numeric(L.A.n, L.A.rp, L.A.ci, L.A.v.p, L.P.rp, L.P.ci, L.P.v.p, L.ap_rp.p, L.ap_ci.p, apv.p,
                       c->flag.p, s, L.ap_narrow && c->opt.setup_kernels == 0);
    amg_spgemm_numeric(L.R.n, L.R.rp, L.R.ci, L.R.v.p, L.ap_rp.p, L.ap_ci.p, apv.p, N.A.rp, N.A.ci, N.A.v.p,
                       c->flag.p, s);
}

// `own` (optional): the buffer holding vals, taken over as the fine level's
// values instead of copying them.  With c->parts set, the operator holds
// several unknowns and is coarsened unknown by unknown.  `feed` (optional):
// publish every level's classical interpolation for a second build.
static void build_hierarchy(Builder *c, Hierarchy &h, const double *vals, DBuf<double> *own = nullptr,
                            LevelFeed *feed = nullptr) {
    hipStream_t s = c->stream;
    const cptr_options &o = c->opt;
    const bool fp32 = (o.precond_precision == CPTR_FP32);
    std::vector<int> parts = c->parts;
    h.L.clear();
    h.L.emplace_back();
    Level &L0 = h.L.back();
    L0.A.n = c->n;
    L0.A.ncols = c->n;
    L0.A.nnz = c->nnzb;
    L0.A.rp = c->rp.p;
    L0.A.ci = c->ci.p;
    if (own && own->p == vals && own->n >= (size_t)c->nnzb) {
        L0.A.v = std::move(*own);
    } else {
        L0.A.v.alloc(c->nnzb);
        CPTR_HIP(hipMemcpyAsync(L0.A.v.p, vals, sizeof(double) * c->nnzb, hipMemcpyDeviceToDevice, s));
    }
    while (true) {
        Level &L = h.L.back();
        const int m = L.A.n;
        L.dinv.alloc(m);
        c->s_d1.alloc(m);   // diagonal of this level
        amg_diag_inv2(m, L.A.rp, L.A.ci, L.A.v.p, o.smoother, L.dinv.p, c->s_d1.p, c->flag.p, s);
        level_bound(c, h, (int)h.L.size() - 1);
        level_vectors(L, m, fp32);
        // (exact sub-solves: the fine level is the coarsest, applied by its
        // dense inverse)
        if (o.exact_subsolves || m <= o.amg_max_coarse || (int)h.L.size() >= o.amg_max_levels) break;
        if (parts.size() > 1) {
            Level nxt;
            if (!coarsen_system(c, L, parts, h.L.size() == 1, nxt)) break;
            h.L.push_back(std::move(nxt));
            continue;
        }
        CsrD &P = L.P;
        SpgPlan pAP;
        int rd[4];
        L.strong.alloc((size_t)L.A.nnz + 1);
        L.cf.alloc((size_t)m + 1);             // state -> C/F
        InterpScratch is;
        const int nc = interp_rows(c, L.A, c->s_d1.p, L.cf.p, L.strong.p, h.L.size() == 1, is, L.P);
        if (nc == 0 || nc == m) break;
        // A P needs only P's row pointers for its plan: P's size and the
        // product's capacity in one read
        spgemm_plan(c, L.A, P, pAP);
        read_ints4(c, P.rp_own.p + m, pAP.off.p + m, pAP.off.p + m + 1, pAP.off.p + m + 2, rd);
        P.nnz = rd[0];
        const int capAP = rd[1], maxAP = rd[2], shapeAP = rd[3];
        compact_interp(c, is, P);
        L.nc = nc;
        if (feed && h.L.size() == 1) {
            LevelFeed::Item it;
            it.n = m;
            it.nc = nc;
            it.cf = L.cf.p;
            it.P = LevelFeed::view(P);
            it.annz = L.A.nnz;
            it.av = L.A.v.p;
            it.dinv = L.dinv.p;
            it.strong = L.strong.p;
            feed->publish(it, s, true);
        }
        csr_transpose(c, P, L.R);
        CsrD AP;
        spgemm_compute(c, L.A, P, pAP, capAP, maxAP, AP, shapeAP);
        // R (A P) needs only A P's row pointers for its plan
        SpgPlan pRAP;
        spgemm_plan(c, L.R, AP, pRAP);
        read_ints3(c, AP.rp_own.p + m, pRAP.off.p + nc, pRAP.off.p + nc + 1, rd);
        spgemm_finish(c, pAP, rd[0], AP);
        Level nxt;
        spgemm_compute(c, L.R, AP, pRAP, rd[1], rd[2], nxt.A);
        spgemm_finish(c, pRAP, read_scalar(nxt.A.rp_own.p + nc, s), nxt.A);
        // A P's pattern, for refreshing this product on new values
        L.ap_rp = std::move(AP.rp_own);
        L.ap_ci = std::move(AP.ci_own);
        L.ap_nnz = AP.nnz;
        L.ap_narrow = (shapeAP == 0);
        if (feed) {
            LevelFeed::Item it;
            it.n = m;
            it.nc = nc;
            it.cf = L.cf.p;
            it.P = LevelFeed::view(P);
            it.R = LevelFeed::view(L.R);
            it.AP = {m, nc, L.ap_nnz, L.ap_rp.p, L.ap_ci.p, nullptr};
            it.Anext = {nxt.A.n, nxt.A.ncols, nxt.A.nnz, nxt.A.rp, nxt.A.ci, nullptr};
            it.ap_narrow = L.ap_narrow;
            feed->publish(it, s, false);
        }
        h.L.push_back(std::move(nxt));
    }
    if (feed) feed->close();
    read_bounds(c, h);
    coarse_inverse(c, h);
    hierarchy_fp32(c, h);
    CPTR_HIP(hipStreamSynchronize(s));
    h.built = true;
}

// The learned counterpart of a classical build that publishes its levels on
// `feed`: the fine level with the classical C/F split and interpolation
// pattern, the learned weights and R_0 = P_0^T; below it the classical
// build's C/F splits and transfer operators (copied as each level is
// published), with every Galerkin product A_{l+1} = R_l A_l P_l formed from
// this hierarchy's own finer level on the classical product's pattern (the
// patterns depend only on the operands' patterns, which are the classical
// ones), then its smoother diagonals, bounds and coarsest inverse.  It runs
// on c's stream, level by level behind the classical build.  Empty when the
// classical build forms no interpolation.
static void build_learned_hierarchy(Builder *c, Hierarchy &h, const float *mlp, LevelFeed &feed) {
    hipStream_t s = c->stream;
    const cptr_options &o = c->opt;
    const bool fp32 = (o.precond_precision == CPTR_FP32);
    h.L.clear();
    LevelFeed::Item it;
    if (!feed.wait_fine(it)) return;
    CPTR_HIP(hipStreamWaitEvent(s, it.ev, 0));
    h.L.emplace_back();
    {
        Level &L0 = h.L.back();
        L0.A.n = L0.A.ncols = it.n;
        L0.A.nnz = it.annz;
        L0.A.rp = c->rp.p;
        L0.A.ci = c->ci.p;
        L0.A.v.alloc(it.annz);
        CPTR_HIP(hipMemcpyAsync(L0.A.v.p, it.av, sizeof(double) * it.annz, hipMemcpyDeviceToDevice, s));
        L0.dinv.alloc(it.n);
        CPTR_HIP(hipMemcpyAsync(L0.dinv.p, it.dinv, sizeof(double) * it.n, hipMemcpyDeviceToDevice, s));
        L0.strong.alloc((size_t)it.annz + 1);
        CPTR_HIP(hipMemcpyAsync(L0.strong.p, it.strong, (size_t)it.annz, hipMemcpyDeviceToDevice, s));
        L0.nc = it.nc;
        L0.cf.alloc((size_t)it.n + 1);
        CPTR_HIP(hipMemcpyAsync(L0.cf.p, it.cf, sizeof(int) * it.n, hipMemcpyDeviceToDevice, s));
        copy_csr(s, it.P, L0.P);
        level_bound(c, h, 0);
        level_vectors(L0, it.n, fp32);
        apply_learned(s, L0, mlp);
        csr_transpose(c, L0.P, L0.R);
    }
    for (size_t l = 0;; ++l) {
        // the classical level l's products, or none (then this level is the
        // coarsest, as it is there)
        if (!feed.wait(l, it)) break;
        CPTR_HIP(hipStreamWaitEvent(s, it.ev, 0));
        Level &L = h.L[l];
        if (l > 0) {
            L.nc = it.nc;
            L.cf.alloc((size_t)L.A.n + 1);
            CPTR_HIP(hipMemcpyAsync(L.cf.p, it.cf, sizeof(int) * L.A.n, hipMemcpyDeviceToDevice, s));
            copy_csr(s, it.P, L.P);
            copy_csr(s, it.R, L.R);
        }
        L.ap_nnz = it.AP.nnz;
        L.ap_narrow = it.ap_narrow;
        L.ap_rp.alloc((size_t)it.AP.n + 1);
        L.ap_ci.alloc((size_t)it.AP.nnz + 1);
        CPTR_HIP(hipMemcpyAsync(L.ap_rp.p, it.AP.rp, sizeof(int) * (it.AP.n + 1), hipMemcpyDeviceToDevice, s));
        if (it.AP.nnz)
            CPTR_HIP(hipMemcpyAsync(L.ap_ci.p, it.AP.ci, sizeof(int) * it.AP.nnz, hipMemcpyDeviceToDevice, s));
        Level nxt;
        copy_csr(s, it.Anext, nxt.A, false);
        galerkin_numeric(c, L, nxt);
        h.L.push_back(std::move(nxt));
        Level &N = h.L.back();
        const int m = N.A.n;
        N.dinv.alloc(m);
        c->s_d1.alloc(m);
        amg_diag_inv2(m, N.A.rp, N.A.ci, N.A.v.p, o.smoother, N.dinv.p, c->s_d1.p, c->flag.p, s);
        level_bound(c, h, (int)l + 1);
        level_vectors(N, m, fp32);
    }
    read_bounds(c, h);
    coarse_inverse(c, h);
    hierarchy_fp32(c, h);
    CPTR_HIP(hipStreamSynchronize(s));
    h.built = true;
}

// Reuse of a hierarchy for new level-0 values on the same pattern (a Newton
// sequence): the C/F splits and the interpolation / restriction operators of
// every level are kept; the Galerkin products A_{l+1} = R_l A_l P_l, the
// smoother diagonals and the coarsest inverse are recomputed from the new
// values with the same kernels as a full setup.
static void refresh_hierarchy(Builder *c, Hierarchy &h, const double *vals, DBuf<double> *own) {
    hipStream_t s = c->stream;
    const cptr_options &o = c->opt;
    if (!h.built || h.L.empty()) throw Error(CPTR_E_STATE, "no hierarchy to reuse");
    Level &L0 = h.L[0];
    if (own && own->p == vals && own->n >= (size_t)c->nnzb)
        L0.A.v = std::move(*own);
    else
        CPTR_HIP(hipMemcpyAsync(L0.A.v.p, vals, sizeof(double) * c->nnzb, hipMemcpyDeviceToDevice, s));
    for (size_t l = 0; l < h.L.size(); ++l) {
        Level &L = h.L[l];
        const int m = L.A.n;
        c->s_d1.alloc(m);
        amg_diag_inv2(m, L.A.rp, L.A.ci, L.A.v.p, o.smoother, L.dinv.p, c->s_d1.p, c->flag.p, s);
        level_bound(c, h, (int)l);
        if (l + 1 == h.L.size()) break;
        if (L.ap_nnz >= 0) {
            // the products on their kept patterns
            galerkin_numeric(c, L, h.L[l + 1]);
        } else {
            CsrD AP, Ac;
            csr_spgemm(c, L.A, L.P, AP);
            csr_spgemm(c, L.R, AP, Ac);
            h.L[l + 1].A = std::move(Ac);
        }
    }
    read_bounds(c, h);
    coarse_inverse(c, h);
    hierarchy_fp32(c, h);
    CPTR_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// V-cycle (zero initial guess); input h.L[lvl].b, returns the buffer holding x
// ---------------------------------------------------------------------------
template <class T> struct Prec;
template <> struct Prec<double> {
    static const double *v(const CsrD &A) { return A.v.p; }
    static double *x(Level &L) { return L.x.p; }
    static double *b(Level &L) { return L.b.p; }
    static double *r(Level &L) { return L.r.p; }
    static const double *dinv(const Level &L) { return L.dinv.p; }
};
template <> struct Prec<float> {
    static const float *v(const CsrD &A) { return A.v32.p; }
    static float *x(Level &L) { return L.x32.p; }
    static float *b(Level &L) { return L.b32.p; }
    static float *r(Level &L) { return L.r32.p; }
    static const float *dinv(const Level &L) { return L.dinv32.p; }
};

// One Chebyshev iteration of the given degree on A x = b, in place on x (from
// zero when `zero`), over [lam/30, 1.1 lam] of the spectrum of D^{-1} A with
// lam the level's Gershgorin bound; r and d[0], d[1] are work vectors
template <class T>
static void cheb_smooth(const Level &L, const T *v, const T *dinv, const T *b, T *x, bool zero, int degree, T *r,
                        T *const *d, hipStream_t s) {
    const int n = L.A.n;
    if (degree == 0) {
        if (zero) CPTR_HIP(hipMemsetAsync(x, 0, sizeof(T) * n, s));
        return;
    }
    const double lmax = 1.1 * L.lam_max, lmin = L.lam_max / 30.0;
    const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    vc_cheb_init<T>(n, L.A.nnz, L.A.rp, L.A.ci, v, dinv, b, zero ? nullptr : x, x, r, d[0], (T)theta, s);
    int cur = 0;
    for (int k = 0; k < degree; ++k) {
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        const double c1 = rho_new * rho, c2 = 2.0 * rho_new / delta;
        vc_cheb_step<T>(n, L.A.nnz, L.A.rp, L.A.ci, v, dinv, d[cur], x, r, d[1 - cur], (T)c1, (T)c2, s);
        cur = 1 - cur;
        rho = rho_new;
    }
}

// the level's five planes in precision T (null when the level has none:
// the sweeps then run on its CSR rows)
template <class T>
static const T *planes(const Level &L) {
    if (L.ell_nx <= 0) return nullptr;
    if constexpr (std::is_same<T, float>::value) return L.ell32.p; else return L.ell64.p;
}
// the level's Jacobi sweeps: on the five planes when the level has them in
// this precision (fine level on the 5-point grid pattern), else on its CSR rows
template <class T>
static void lv_presmooth(const Level &L, const T *v, const T *dinv, T omega, const T *b, T *x, T *r, hipStream_t s) {
    if (const T *e = planes<T>(L)) return vc_ell5_presmooth_residual<T>(L.A.n, L.ell_nx, e, dinv, omega, b, x, r, s);
    vc_presmooth_residual<T>(L.A.n, L.A.nnz, L.A.rp, L.A.ci, v, dinv, omega, b, x, r, s);
}
template <class T>
static void lv_sweep(const Level &L, const T *v, const T *dinv, T omega, const T *b, const T *x, const T *r, T *xout,
                     T *rout, hipStream_t s) {
    if (const T *e = planes<T>(L))
        return vc_ell5_sweep_residual<T>(L.A.n, L.ell_nx, e, dinv, omega, b, x, r, xout, rout, s);
    vc_sweep_residual<T>(L.A.n, L.A.nnz, L.A.rp, L.A.ci, v, dinv, omega, b, x, r, xout, rout, s);
}
template <class T>
static void lv_smooth(const Level &L, const T *v, const T *dinv, T omega, const T *b, const T *xin, T *xout,
                      hipStream_t s) {
    if (const T *e = planes<T>(L)) return vc_ell5_smooth<T>(L.A.n, L.ell_nx, e, dinv, omega, b, xin, xout, s);
    vc_smooth<T>(L.A.n, L.A.nnz, L.A.rp, L.A.ci, v, dinv, omega, b, xin, xout, s);
}

template <class T>
static T *vcycle(cptr_ctx *c, Hierarchy &h, int lvl, hipStream_t s) {
    Level &L = h.L[lvl];
    const int n = L.A.n;
    T *x = Prec<T>::x(L);
    T *b = Prec<T>::b(L);
    if (lvl == (int)h.L.size() - 1) {
        if (h.bt) {
            const BlockTri &bt = *h.bt;
            bt_solve<T>(bt.ng, bt.g, L.A.rp, L.A.ci, L.A.v.p, bt.perm.p, bt.rowof.p, bt.Sinv.p, bt.G.p, bt.z.p,
                        bt.xw.p, b, x, s);
        } else if constexpr (std::is_same<T, double>::value) {
            vc_dense_apply<double>(n, h.cinv.p, b, x, s);
        } else {
            vc_dense_apply_mixed(n, h.cinv.p, b, x, s);
        }
        return x;
    }
    const cptr_options &o = c->opt;
    const T omega = (T)((o.smoother == CPTR_SMOOTH_JACOBI) ? o.jacobi_omega : 1.0);
    const T *v = Prec<T>::v(L.A);
    const T *dinv = Prec<T>::dinv(L);
    // buffers: x (the level's result) and three spares of the same length
    T *const X = x;
    T *spare[3] = {Prec<T>::r(L), Prec<T>::r(L) + n, Prec<T>::r(L) + 2 * (size_t)n};
    if (o.smoother == CPTR_SMOOTH_CHEBYSHEV) {
        // Chebyshev smoothing before and after the coarse correction, each one
        // Chebyshev iteration of degree cheb_degree * sweeps, in place on X
        Level &Lc = h.L[lvl + 1];
        T *r = spare[0];
        T *const d[2] = {spare[1], spare[2]};
        cheb_smooth<T>(L, v, dinv, b, X, true, o.cheb_degree * o.pre_sweeps, r, d, s);
        vc_residual<T>(n, L.A.nnz, L.A.rp, L.A.ci, v, b, X, r, s);
        vc_spmv<T>(L.R.n, L.R.nnz, L.R.rp, L.R.ci, Prec<T>::v(L.R), r, Prec<T>::b(Lc), s);
        const T *xc = vcycle<T>(c, h, lvl + 1, s);
        vc_prolong_to<T>(n, L.P.nnz, L.P.rp, L.P.ci, Prec<T>::v(L.P), xc, X, X, s);
        cheb_smooth<T>(L, v, dinv, b, X, false, o.cheb_degree * o.post_sweeps, r, d, s);
        return X;
    }
    // pre-smoothing from zero; every further sweep fused with the next residual
    T *xa = X, *ra = spare[0];
    const T *rres = b;   // what is restricted
    if (o.pre_sweeps >= 1) {
        lv_presmooth<T>(L, v, dinv, omega, b, xa, ra, s);
        T *xb = spare[1], *rb = spare[2];
        for (int k = 1; k < o.pre_sweeps; ++k) {
            lv_sweep<T>(L, v, dinv, omega, b, xa, ra, xb, rb, s);
            std::swap(xa, xb);
            std::swap(ra, rb);
        }
        rres = ra;
    } else {
        CPTR_HIP(hipMemsetAsync(xa, 0, sizeof(T) * n, s));
    }
    Level &Ln = h.L[lvl + 1];
    vc_spmv<T>(L.R.n, L.R.nnz, L.R.rp, L.R.ci, Prec<T>::v(L.R), rres, Prec<T>::b(Ln), s);
    const T *xc = vcycle<T>(c, h, lvl + 1, s);
    // prolongation, then post-smoothing ping-ponging so that the last write
    // lands in X: the prolonged value goes to X for an even number of sweeps
    T *Y = (xa == X) ? spare[0] : ((spare[0] != xa) ? spare[0] : spare[1]);
    T *cur = (o.post_sweeps % 2 == 0) ? X : Y;
    T *oth = (cur == X) ? Y : X;
    vc_prolong_to<T>(n, L.P.nnz, L.P.rp, L.P.ci, Prec<T>::v(L.P), xc, xa, cur, s);
    for (int k = 0; k < o.post_sweeps; ++k) {
        lv_smooth<T>(L, v, dinv, omega, b, cur, oth, s);
        std::swap(cur, oth);
    }
    return X;
}

// ---------------------------------------------------------------------------
// multi-stage preconditioner: y = M^{-1} r (Eq. multistageprec; Algorithm 2
// for CPTR3, Algorithm 1 for CPR and for the two-stage CPTR scheme with the
// system AMG on B_ee), r and y double, internals in T
// ---------------------------------------------------------------------------
template <class T>
static void precond_apply(cptr_ctx *c, const double *r, double *y) {
    hipStream_t s = c->stream;
    const int n = c->n, b = c->b;
    const bool f32 = std::is_same<T, float>::value;
    const T *abar = f32 ? (const T *)c->abar32.p : (const T *)c->abar.p;
    const T *dinv = f32 ? (const T *)c->dinv32.p : (const T *)c->dinv.p;
    const T *slabT = f32 ? (const T *)c->slabT32.p : (const T *)c->slabT.p;
    const T *slabP = f32 ? (const T *)c->slabP32.p : (const T *)c->slabP.p;
    T *tw = f32 ? (T *)c->tw32.p : (T *)c->tw.p;
    const T *xT = nullptr, *vP = nullptr;
    const int variant = c->opt.variant;
    if (variant == CPTR_VARIANT_CPTR3) {
        const bool t_first = (c->opt.stage_order == CPTR_T_THEN_P);
        Hierarchy &h1 = c->H[t_first ? 0 : 1];
        Hierarchy &h2 = c->H[t_first ? 1 : 0];
        const int comp1 = t_first ? c->it : c->ip, comp2 = t_first ? c->ip : c->it;
        // M1: gather, V-cycle
        ms_stage_input<T>(n, b, c->rp.p, c->ci.p, (const T *)nullptr, comp1, r, (const T *)nullptr,
                          Prec<T>::b(h1.L[0]), s);
        const T *x1 = vcycle<T>(c, h1, 0, s);
        c->mark(1);
        // M2 on z = r - Abar x (only its comp2 entries are needed)
        const T *cpl = f32 ? (const T *)c->cpl32.p : (const T *)c->cpl.p;
        ms_stage_input<T>(n, b, c->rp.p, c->ci.p, cpl, comp2, r, x1, Prec<T>::b(h2.L[0]), s);
        const T *x2 = vcycle<T>(c, h2, 0, s);
        c->mark(2);
        xT = t_first ? x1 : x2;
        vP = t_first ? x2 : x1;
    } else if (variant == CPTR_VARIANT_CPR) {
        Hierarchy &hp = c->H[1];
        ms_stage_input<T>(n, b, c->rp.p, c->ci.p, (const T *)nullptr, c->ip, r, (const T *)nullptr,
                          Prec<T>::b(hp.L[0]), s);
        vP = vcycle<T>(c, hp, 0, s);
        c->mark(1);
        c->mark(2);
    } else if (variant == CPTR_VARIANT_CPTR) {
        // two-stage CPTR: one system V-cycle on [r_P; r_T]; the last stage
        // takes its P half as the P correction and its T half as the T one
        Hierarchy &h = c->H[0];
        T *bs = Prec<T>::b(h.L[0]);
        ms_stage_input<T>(n, b, c->rp.p, c->ci.p, (const T *)nullptr, c->ip, r, (const T *)nullptr, bs, s);
        ms_stage_input<T>(n, b, c->rp.p, c->ci.p, (const T *)nullptr, c->it, r, (const T *)nullptr, bs + n, s);
        const T *xs = vcycle<T>(c, h, 0, s);
        c->mark(1);
        c->mark(2);
        vP = xs;
        xT = xs + n;
    } else {
        c->mark(1);
        c->mark(2);
    }
    // last stage on u = r - Abar (x + v), combined output y = x + v + ilu^{-1} u
    if (c->use_tiles)
    {
        const T *tb = f32 ? (const T *)c->tb32.p : (const T *)c->tb.p;
        bilu_apply_tiles<T>(c->ts, b, c->rp.p, c->ci.p, abar, tb, dinv, slabT, slabP, c->ip, c->it, r, xT, vP, tw, y,
                            s);
    }
    else
        bj_apply_cells<T>(n, b, c->rp.p, c->ci.p, dinv, slabT, slabP, c->ip, c->it, r, xT, vP, y, s);
}

static void precond(cptr_ctx *c, const double *r, double *y) {
    if (c->opt.precond_precision == CPTR_FP32)
        precond_apply<float>(c, r, y);
    else
        precond_apply<double>(c, r, y);
}

// Asymptotic V-cycle convergence factor of a hierarchy on A e = 0:
// e <- e - V(A e) from a SplitMix64-uniform start in [-1, 1), K cycles,
// rho = (|e_K| / |e_0|)^(1/K), on stream s.  V-cycles in FP64, or with fp32
// the FP32 V-cycle the precision-split preconditioner applies (e and A e in
// FP64, A e rounded to FP32 as the V-cycle's input, its output subtracted in
// FP64).
static double conv_factor(cptr_ctx *c, Hierarchy &h, int cycles, uint64_t seed, hipStream_t s,
                          bool fp32 = false) {
    Level &L0 = h.L[0];
    const int n = L0.A.n;
    DBuf<double> e, part, nrm;
    e.alloc(n);
    const int nblk = kr_nblk(n);
    part.alloc(nblk);
    nrm.alloc(2);
    vc_hash_uniform(n, seed, e.p, s);
    kr_norm2_partial(n, e.p, part.p, nblk, s);
    kr_reduce(part.p, nblk, 1, nrm.p, s);
    for (int k = 0; k < cycles; ++k) {
        if (fp32) {
            vc_spmv_to_float(n, L0.A.rp, L0.A.ci, L0.A.v.p, e.p, L0.b32.p, s);
            const float *x = vcycle<float>(c, h, 0, s);
            vc_sub_float(n, x, e.p, s);
        } else {
            vc_spmv<double>(n, L0.A.nnz, L0.A.rp, L0.A.ci, L0.A.v.p, e.p, L0.b.p, s);
            const double *x = vcycle<double>(c, h, 0, s);
            vc_sub(n, x, e.p, s);
        }
    }
    kr_norm2_partial(n, e.p, part.p, nblk, s);
    kr_reduce(part.p, nblk, 1, nrm.p + 1, s);
    double v[2];
    read_bytes(v, nrm.p, 2 * sizeof(double), s);
    if (!(v[0] > 0.0)) return 0.0;
    return std::pow(std::sqrt(v[1]) / std::sqrt(v[0]), 1.0 / cycles);
}

constexpr int RHO_CYCLES = 10;
constexpr int MAX_REUSE_BACKOFF = 8;
constexpr uint64_t RHO_SEED = 0;

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
static void validate_options(const cptr_options &o) {
    if (o.variant != CPTR_VARIANT_CPTR3 && o.variant != CPTR_VARIANT_CPR && o.variant != CPTR_VARIANT_CPTR &&
        o.variant != CPTR_VARIANT_LAST_ONLY)
        throw Error(CPTR_E_ARG, "unknown variant");
    if (o.restart < 1 || o.restart > 200) throw Error(CPTR_E_ARG, "restart must be 1..200");
    if (o.max_iters < 1) throw Error(CPTR_E_ARG, "max_iters must be positive");
    if (!(o.rtol > 0.0)) throw Error(CPTR_E_ARG, "rtol must be positive");
    if (o.precond_precision == CPTR_FP32 && o.krylov != CPTR_FGMRES)
        throw Error(CPTR_E_ARG, "the FP32 preconditioner needs flexible GMRES");
    if (o.amg_max_coarse < 1 || o.amg_max_levels < 1) throw Error(CPTR_E_ARG, "AMG size limits must be positive");
    if (o.ilu_tile_x < 1 || o.ilu_tile_y < 1) throw Error(CPTR_E_ARG, "ILU tile must be at least 1 x 1");
    if (o.pre_sweeps < 0 || o.post_sweeps < 0) throw Error(CPTR_E_ARG, "negative smoothing sweeps");
    if (o.setup_kernels < 0 || o.setup_kernels > 3) throw Error(CPTR_E_ARG, "setup_kernels must be 0, 1, 2 or 3");
    if (o.exact_subsolves < 0 || o.exact_subsolves > 2) throw Error(CPTR_E_ARG, "exact_subsolves must be 0, 1 or 2");
    if (o.smoother < CPTR_SMOOTH_JACOBI || o.smoother > CPTR_SMOOTH_CHEBYSHEV) throw Error(CPTR_E_ARG, "unknown smoother");
    if (o.smoother == CPTR_SMOOTH_CHEBYSHEV && (o.cheb_degree < 1 || o.cheb_degree > 16))
        throw Error(CPTR_E_ARG, "cheb_degree must be 1..16");
    if (o.t_interp < CPTR_INTERP_CLASSICAL || o.t_interp > CPTR_INTERP_LEARNED_FORCED)
        throw Error(CPTR_E_ARG, "unknown t_interp");
    if (o.stop_unscaled != 0 && o.stop_unscaled != 1) throw Error(CPTR_E_ARG, "stop_unscaled must be 0 or 1");
    if (o.judge_cycles < 1 || o.judge_cycles > 1000) throw Error(CPTR_E_ARG, "judge_cycles must be 1..1000");
    if (o.t_interp != CPTR_INTERP_CLASSICAL && (o.amg_pmax < 1 || o.amg_pmax > 16))
        throw Error(CPTR_E_ARG, "learned interpolation needs amg_pmax in 1..16");
}

// A full build of hierarchy k.  For the temperature stage with learned
// interpolation requested, the classical and the learned hierarchies are both
// built and the learned one is kept only if its measured V-cycle convergence
// factor is lower (CPTR_INTERP_LEARNED_FORCED keeps it without the judge).
static void full_build(cptr_ctx *c, Builder &B, int k, const double *vals, DBuf<double> *own, Hierarchy &dst) {
    const bool learned = (k == 0) && c->opt.variant == CPTR_VARIANT_CPTR3 && c->have_mlp &&
                         c->opt.t_interp != CPTR_INTERP_CLASSICAL;
    if (k == 0) {
        c->used_learned = 0;
        c->rho_cls = c->rho_lrn = -1.0;
    }
    if (!learned) {
        build_hierarchy(&B, dst, vals, own);
        return;
    }
    const bool judge = (c->opt.t_interp == CPTR_INTERP_LEARNED);
    // the learned hierarchy (and its convergence factor) on its own stream
    // and host thread, level by level behind the classical build, whose C/F
    // splits and transfer operators it keeps below the fine level (the
    // learned correction changes only the fine level's weights)
    Hierarchy hl;
    double rl = -1.0;
    std::exception_ptr err;
    Builder &B2 = c->bld[2];
    B2.stream = c->side[2];
    B2.opt = B.opt;
    B2.n = B.n;
    B2.gx = B.gx;
    B2.gy = B.gy;
    B2.ell_nx = B.ell_nx;
    B2.nnzb = B.nnzb;
    B2.rp.p = B.rp.p;
    B2.ci.p = B.ci.p;
    LevelFeed feed;
    const bool fp32 = (c->opt.precond_precision == CPTR_FP32);
    std::thread t2([c, &B2, &hl, &rl, &err, &feed, judge, fp32]() {
        try {
            CPTR_HIP(hipSetDevice(c->device));
            StreamScope scope(B2.stream);
            if (!B2.flag.p) {
                B2.flag.alloc(4);
                fill_int(B2.flag.p, 0, 1, B2.stream);
            }
            build_learned_hierarchy(&B2, hl, c->mlp.p, feed);
            if (judge && hl.L.size() > 1) rl = conv_factor(c, hl, c->opt.judge_cycles, RHO_SEED, B2.stream, fp32);
        } catch (...) {
            err = std::current_exception();
        }
    });
    std::exception_ptr err1;
    double rc = -1.0;
    try {
        build_hierarchy(&B, dst, vals, own, &feed);
        if (judge && dst.L.size() > 1) rc = conv_factor(c, dst, c->opt.judge_cycles, RHO_SEED, B.stream, fp32);
    } catch (...) {
        err1 = std::current_exception();
        feed.close();
    }
    t2.join();
    if (err1) std::rethrow_exception(err1);
    if (err) std::rethrow_exception(err);
    if (dst.L.size() < 2 || hl.L.size() < 2) return;   // a single level: no interpolation to learn
    if (!judge || rl < rc) {
        dst = std::move(hl);
        c->used_learned = 1;
    }
    c->rho_cls = rc;
    c->rho_lrn = rl;
}

static double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

static void do_setup_values(cptr_ctx *c, const double *vals, bool reuse) {
    hipStream_t s = c->stream;
    const auto t_start = std::chrono::steady_clock::now();
    const int n = c->n, b = c->b, nnzb = c->nnzb;
    const bool fp32 = (c->opt.precond_precision == CPTR_FP32);
    const bool sys = (c->opt.variant == CPTR_VARIANT_CPTR);
    c->abar.alloc((size_t)nnzb * b * b);
    c->wp.alloc((size_t)n * b);
    c->wt.alloc((size_t)n * b);
    c->beta.alloc(n);
    // s_i4[0]: the lowest singular cell of the decoupling; s_i4[1]: the
    // non-finite flag of the values (both come back in one read).  CPTR3 and
    // CPR check the values inside phase 1, which reads every block row; the
    // other variants scan them on a side stream beside it
    c->s_i4.alloc(2);
    fill_int(c->s_i4.p, 0x7fffffff, 1, s);
    fill_int(c->s_i4.p + 1, 0, 1, s);
    const bool rows_kernel = !sys && c->opt.variant != CPTR_VARIANT_LAST_ONLY;
    if (!rows_kernel) {
        CPTR_HIP(hipEventRecord(c->ev_side[2], s));
        CPTR_HIP(hipStreamWaitEvent(c->side[2], c->ev_side[2], 0));
        count_nonfinite(vals, (size_t)nnzb * b * b, c->s_i4.p + 1, c->side[2]);
        CPTR_HIP(hipEventRecord(c->ev_side[2], c->side[2]));
    }
    c->slabT.alloc((size_t)nnzb * b);
    c->slabP.alloc((size_t)nnzb * b);
    DBuf<double> &ctt = c->ctt, &bpp = c->bpp;
    ctt.alloc(nnzb);
    bpp.alloc(nnzb);
    if (fp32) {
        c->abar32.alloc((size_t)nnzb * b * b);
        c->slabT32.alloc((size_t)nnzb * b);
        c->slabP32.alloc((size_t)nnzb * b);
    }
    if (c->opt.variant == CPTR_VARIANT_LAST_ONLY) {
        CPTR_HIP(hipMemcpyAsync(c->abar.p, vals, sizeof(double) * nnzb * b * b, hipMemcpyDeviceToDevice, s));
        launch_extract(n, b, nnzb, c->abar.p, c->ip, c->it, ctt.p, bpp.p, c->slabT.p, c->slabP.p,
                       fp32 ? c->abar32.p : nullptr, fp32 ? c->slabT32.p : nullptr, fp32 ? c->slabP32.p : nullptr, s);
    } else if (sys) {
        // phase 1: the weights and the elliptic block B_ee (all the system
        // AMG setup needs)
        if ((size_t)4 * nnzb > 0x7fffffffULL) throw Error(CPTR_E_ARG, "elliptic block exceeds 32-bit indexing");
        c->ee_rp.alloc(2 * (size_t)n + 1);
        c->ee_ci.alloc(4 * (size_t)nnzb);
        c->ee_v.alloc(4 * (size_t)nnzb);
        launch_decouple_weights(c->opt.variant, n, b, c->rp.p, c->ci.p, vals, c->ip, c->it, c->wp.p, c->wt.p,
                                c->beta.p, c->s_i4.p, nullptr, nullptr, c->ee_rp.p, c->ee_ci.p, c->ee_v.p, s);
    } else {
        // phase 1: the weights and the two scalar operators (all the AMG setups need)
        launch_decouple_weights_rows(c->opt.variant, n, b, c->rp.p, c->ci.p, vals, c->ip, c->it, c->wp.p, c->wt.p,
                                     c->beta.p, c->s_i4.p, c->s_i4.p + 1, ctt.p, bpp.p, s);
    }
    if (!rows_kernel) CPTR_HIP(hipStreamWaitEvent(s, c->ev_side[2], 0));
    int chk[2];
    read_bytes(chk, c->s_i4.p, 2 * sizeof(int), s);
    if (chk[1] & 16) throw Error(CPTR_E_NONFINITE, "non-finite matrix entry");
    int bad = chk[0];
    if (bad != 0x7fffffff)
        throw Error(CPTR_E_SINGULAR_BLOCK, "singular decoupling block (D_ss or Ahat_PP) in cell " + std::to_string(bad));
    // scalar stages: the two hierarchies are built concurrently, each on its
    // own stream and host thread, while this stream factors the last stage
    c->tph[0] = ms_since(t_start);
    const auto t_hier = std::chrono::steady_clock::now();
    // (slot 0 holds the system hierarchy of B_ee for the two-stage scheme,
    // which is always built anew)
    const bool need[2] = {c->opt.variant == CPTR_VARIANT_CPTR3 || sys,
                          c->opt.variant == CPTR_VARIANT_CPTR3 || c->opt.variant == CPTR_VARIANT_CPR};
    const double *svals[2] = {sys ? c->ee_v.p : ctt.p, bpp.p};
    bool refresh[2] = {false, false};
    for (int k = 0; k < 2; ++k) {
        refresh[k] = need[k] && reuse && c->H[k].built && !sys;
        if (!reuse) {
            c->skip_left[k] = 0;
            c->backoff[k] = 1;
        } else if (refresh[k] && c->skip_left[k] > 0) {
            --c->skip_left[k];
            refresh[k] = false;
        }
    }
    std::atomic<int> kept{0};
    c->reused = 0;
    c->rho[0] = c->rho[1] = -1.0;
    CPTR_HIP(hipEventRecord(c->ev_dec, s));
    std::exception_ptr err[2];
    std::thread th[2];
    for (int k = 0; k < 2; ++k) {
        if (!need[k]) continue;
        Builder &B = c->bld[k];
        B.stream = c->side[k];
        B.opt = c->opt;
        const bool ee = sys && k == 0;
        B.n = ee ? 2 * n : n;
        B.nnzb = ee ? 4 * nnzb : nnzb;
        B.rp.p = ee ? c->ee_rp.p : c->rp.p;
        B.ci.p = ee ? c->ee_ci.p : c->ci.p;
        B.parts.clear();
        B.aux = nullptr;
        B.device = c->device;
        B.gx = c->nx;
        B.gy = c->ny;
        B.ell_nx = (!ee && c->ell5) ? c->nx : 0;
        if (ee) {
            B.parts = {n, n};
            // the pressure builder is idle in the two-stage scheme: it
            // coarsens the temperature block of every level concurrently
            Builder &A2 = c->bld[1];
            A2.stream = c->side[1];
            A2.opt = c->opt;
            A2.device = c->device;
            A2.parts.clear();
            A2.aux = nullptr;
            B.aux = &A2;
        }
        c->tph[1 + k] = 0.0;
        th[k] = std::thread([c, k, sys, fp32, &B, &svals, &err, &refresh, &kept, t_hier]() {
            try {
                CPTR_HIP(hipSetDevice(c->device));
                StreamScope scope(B.stream);
                if (!B.flag.p) {
                    B.flag.alloc(4);
                    fill_int(B.flag.p, 0, 1, B.stream);
                }
                CPTR_HIP(hipStreamWaitEvent(B.stream, c->ev_dec, 0));
                // the fine level takes over the buffer of its values
                DBuf<double> *own = k == 0 ? (sys ? &c->ee_v : &c->ctt) : &c->bpp;
                if (refresh[k] && c->backoff[k] > 1) {
                    // the hierarchy's last trial failed: its trial (refresh
                    // and measurement, on the trial stream and a thread of
                    // its own) runs beside a speculative rebuild, and the
                    // decision then keeps one of the two -- the same choice,
                    // and the same hierarchies, as trying first
                    Builder &BT = c->bld_trial;
                    BT.stream = c->side_trial;
                    BT.opt = B.opt;
                    BT.n = B.n;
                    BT.nnzb = B.nnzb;
                    BT.rp.p = B.rp.p;
                    BT.ci.p = B.ci.p;
                    BT.parts = B.parts;
                    BT.aux = nullptr;
                    BT.device = c->device;
                    BT.gx = B.gx;
                    BT.gy = B.gy;
                    BT.ell_nx = B.ell_nx;
                    const int prev_used = c->used_learned;
                    double rho_t = -1.0;
                    std::exception_ptr terr;
                    std::thread tt([c, k, fp32, &BT, &svals, &rho_t, &terr]() {
                        try {
                            CPTR_HIP(hipSetDevice(c->device));
                            StreamScope scope2(BT.stream);
                            if (!BT.flag.p) {
                                BT.flag.alloc(4);
                                fill_int(BT.flag.p, 0, 1, BT.stream);
                            }
                            CPTR_HIP(hipStreamWaitEvent(BT.stream, c->ev_dec, 0));
                            refresh_hierarchy(&BT, c->H[k], svals[k], nullptr);
                            rho_t = conv_factor(c, c->H[k], RHO_CYCLES, RHO_SEED, BT.stream, fp32);
                        } catch (...) {
                            terr = std::current_exception();
                        }
                    });
                    struct Join {
                        std::thread &t;
                        ~Join() { if (t.joinable()) t.join(); }
                    } join_tt{tt};
                    Hierarchy hn;
                    full_build(c, B, k, svals[k], own, hn);
                    tt.join();
                    if (terr) std::rethrow_exception(terr);
                    c->rho[k] = rho_t;
                    if (rho_t < c->opt.reuse_rho_max) {
                        kept.fetch_or(1 << k);
                        c->backoff[k] = 1;
                        if (k == 0) {
                            c->used_learned = prev_used;
                            c->rho_cls = c->rho_lrn = -1.0;
                        }
                    } else {
                        c->skip_left[k] = c->backoff[k];
                        c->backoff[k] = std::min(2 * c->backoff[k], MAX_REUSE_BACKOFF);
                        c->H[k] = std::move(hn);
                    }
                } else if (refresh[k]) {
                    // reuse decision: keep the refreshed hierarchy while its
                    // measured V-cycle convergence factor stays below the
                    // threshold, else build it anew
                    refresh_hierarchy(&B, c->H[k], svals[k], own);
                    c->rho[k] = conv_factor(c, c->H[k], RHO_CYCLES, RHO_SEED, B.stream, fp32);
                    if (c->rho[k] < c->opt.reuse_rho_max) {
                        kept.fetch_or(1 << k);
                        c->backoff[k] = 1;
                        // a kept temperature hierarchy keeps its interpolation
                        // (used_learned) and is not judged again
                        if (k == 0) c->rho_cls = c->rho_lrn = -1.0;
                    } else {
                        c->skip_left[k] = c->backoff[k];
                        c->backoff[k] = std::min(2 * c->backoff[k], MAX_REUSE_BACKOFF);
                        // hand the values back before the old hierarchy goes
                        *own = std::move(c->H[k].L[0].A.v);
                        full_build(c, B, k, svals[k], own, c->H[k]);
                    }
                } else {
                    full_build(c, B, k, svals[k], own, c->H[k]);
                }
                CPTR_HIP(hipEventRecord(c->ev_side[k], B.stream));
                c->tph[1 + k] = ms_since(t_hier);
            } catch (...) {
                err[k] = std::current_exception();
            }
        });
    }
    struct Joiner {
        std::thread *t;
        ~Joiner() { for (int k = 0; k < 2; ++k) if (t[k].joinable()) t[k].join(); }
    } joiner{th};
    // phase 2 of the scaling, concurrently with the hierarchy builds: the
    // scaled matrix, its column slabs and FP32 copies and the BILU(0)
    // sweeps' in-tile neighbour blocks, then the last stage
    const bool tile_blocks = c->use_tiles && bilu_wave_ok(c->ts, b);
    if (tile_blocks) {
        if (fp32)
            c->tb32.alloc((size_t)n * 4 * b * b);
        else
            c->tb.alloc((size_t)n * 4 * b * b);
    }
    const bool tb_in_apply = tile_blocks && c->opt.variant != CPTR_VARIANT_LAST_ONLY;
    if (c->opt.variant != CPTR_VARIANT_LAST_ONLY)
        launch_decouple_apply(c->opt.variant, n, b, c->rp.p, c->ci.p, vals, c->ip, c->it, c->wp.p, c->wt.p,
                              c->beta.p, c->abar.p, c->slabT.p, c->slabP.p, fp32 ? c->abar32.p : nullptr,
                              fp32 ? c->slabT32.p : nullptr, fp32 ? c->slabP32.p : nullptr, s, c->ts.nx, c->ts.tx,
                              c->ts.ty, tb_in_apply && fp32 ? c->tb32.p : nullptr,
                              tb_in_apply && !fp32 ? c->tb.p : nullptr);
    if (c->opt.variant == CPTR_VARIANT_CPTR3) {
        const bool t_first = (c->opt.stage_order == CPTR_T_THEN_P);
        c->cpl.alloc(nnzb);
        if (fp32) c->cpl32.alloc(nnzb);
        ms_gather_comp(nnzb, b, t_first ? c->slabT.p : c->slabP.p, t_first ? c->ip : c->it, c->cpl.p,
                       fp32 ? c->cpl32.p : nullptr, s);
    }
    c->dinv.alloc((size_t)n * b * b);
    fill_int(c->s_i4.p, 0x7fffffff, 1, s);
    if (c->use_tiles) {
        bilu_factor_tiles(c->ts, n, b, c->rp.p, c->ci.p, c->tpos.p, c->abar.p, c->dinv.p, c->s_i4.p, 0, 0, s);
        bilu_factor_tiles(c->ts, n, b, c->rp.p, c->ci.p, c->tpos.p, c->abar.p, c->dinv.p, c->s_i4.p, 1, 0, s);
    } else {
        bj_factor_cells(n, b, c->rp.p, c->ci.p, c->abar.p, c->dinv.p, c->s_i4.p, nullptr, s);
    }
    // the sweeps' side arrays (without the scaling's apply phase: gathered
    // from the copied matrix), also while the hierarchies are still being built
    if (tile_blocks && !tb_in_apply) {
        if (fp32)
            bilu_tile_blocks<float>(c->ts, n, b, c->rp.p, c->ci.p, c->abar.p, c->tb32.p, s);
        else
            bilu_tile_blocks<double>(c->ts, n, b, c->rp.p, c->ci.p, c->abar.p, c->tb.p, s);
    }
    if (fp32) {
        c->dinv32.alloc((size_t)n * b * b);
        to_float(c->dinv.p, c->dinv32.p, (size_t)n * b * b, s);
        c->tw32.alloc(2 * (size_t)n * b);
    } else {
        c->tw.alloc(2 * (size_t)n * b);
    }
    bad = read_scalar(c->s_i4.p, s);
    for (int k = 0; k < 2; ++k)
        if (th[k].joinable()) th[k].join();
    for (int k = 0; k < 2; ++k)
        if (err[k]) {
            // a failed build may leave work queued on the side streams that
            // reads the context's arrays: it ends before the error returns
            for (int j = 0; j < 3; ++j) (void)hipStreamSynchronize(c->side[j]);
            std::rethrow_exception(err[k]);
        }
    c->reused = kept.load();
    for (int k = 0; k < 2; ++k)
        if (need[k]) CPTR_HIP(hipStreamWaitEvent(s, c->ev_side[k], 0));
    if (bad != 0x7fffffff)
        throw Error(CPTR_E_SINGULAR_BLOCK, "singular ILU pivot block in cell " + std::to_string(bad));
    CPTR_HIP(hipStreamSynchronize(s));
    c->tph[3] = ms_since(t_start);
}

static void alloc_krylov(cptr_ctx *c) {
    const size_t N = (size_t)c->n * c->b;
    const int m = c->opt.restart;
    c->V.alloc((m + 1) * N);
    c->Z.alloc(m * N);
    c->w.alloc(N);
    c->x.alloc(N);
    c->rhsbar.alloc(N);
    c->r.alloc(N);
    c->tmpv.alloc(N);
    const int nblk = kr_nblk((int)N);
    c->part.alloc((size_t)nblk * (m + 2));
    c->part2.alloc((size_t)nblk * (m + 2));
    c->hcol.alloc(m + 2);
    c->hcol2.alloc(m + 2);
    c->Hm.alloc((size_t)(m + 1) * m);
    c->cs.alloc(m);
    c->sn.alloc(m);
    c->g.alloc(m + 1);
    c->y.alloc(m);
    c->scal.alloc(2);
    c->hinfo.alloc(4);
    if (!c->hinfo_host) CPTR_HIP(hipHostMalloc((void **)&c->hinfo_host, 8 * sizeof(double), hipHostMallocDefault));
    c->m_alloc = m;
}

// ---------------------------------------------------------------------------
// restarted right-preconditioned GMRES / FGMRES on Abar x = bbar
// ---------------------------------------------------------------------------
static double device_norm(cptr_ctx *c, const double *v, int N) {
    const int nblk = kr_nblk(N);
    kr_norm2_partial(N, v, c->part.p, nblk, c->stream);
    kr_reduce(c->part.p, nblk, 1, c->hcol.p, c->stream);
    return std::sqrt(read_scalar(c->hcol.p, c->stream));
}

// |b - A x| from the scaled residual rbar = bbar - Abar x: the unscaled
// residual is N rbar with N the inverse of the per-cell left scaling.
static double unscaled_norm(cptr_ctx *c, const double *rbar) {
    const int N = c->n * c->b;
    if (c->opt.variant == CPTR_VARIANT_LAST_ONLY)
        return device_norm(c, rbar, N);
    launch_unscale(c->opt.variant, c->n, c->b, rbar, c->ip, c->it, c->wp.p, c->wt.p, c->beta.p, c->tmpv.p,
                   c->stream);
    return device_norm(c, c->tmpv.p, N);
}

// Restarted (F)GMRES on the scaled system.  bnorm0 > 0 with the option
// stop_unscaled: the solve also requires |b - A x| <= rtol |b| (bnorm0 =
// |b|); after a cycle that ends above it, later cycles stop their Givens
// estimate at min(target, |rbar| (rtol |b| / |b - A x|) / 2).
static cptr_status run_gmres(cptr_ctx *c, cptr_result *res, double bnorm0) {
    hipStream_t s = c->stream;
    const int N = c->n * c->b;
    const int m = c->opt.restart;
    const size_t ld = (size_t)N;
    const int nblk = kr_nblk(N);
    c->history.clear();
    for (double &t : c->tacc) t = 0.0;
    c->tsteps = 0;
    const double bnorm = device_norm(c, c->rhsbar.p, N);
    fill_double(c->x.p, 0.0, N, s);
    if (bnorm == 0.0) {
        res->iterations = 0;
        res->converged = 1;
        res->rel_res_scaled = 0.0;
        return CPTR_OK;
    }
    CPTR_HIP(hipMemcpyAsync(c->r.p, c->rhsbar.p, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    int its = 0, restarts = 0;
    double true_rel = 1.0;
    bool converged = false;
    double target = c->opt.rtol * bnorm;
    const bool unscaled = c->opt.stop_unscaled && bnorm0 > 0.0;
    while (true) {
        kr_norm2_partial(N, c->r.p, c->part.p, nblk, s);
        kr_cycle_prep(c->part.p, nblk, m, c->g.p, c->scal.p, c->hinfo.p, s);
        kr_scale(N, c->r.p, c->scal.p, c->V.p, s);
        int k = 0;
        bool breakdown = false;
        for (int j = 0; j < m; ++j) {
            double *vj = c->V.p + (size_t)j * ld;
            double *zj = c->Z.p + (size_t)j * ld;
            c->mark(0);
            precond(c, vj, zj);
            c->mark(3);
            launch_bsr_spmv(c->n, c->b, c->rp.p, c->ci.p, c->abar.p, zj, c->w.p, s);
            c->mark(4);
            kr_mdot(N, j + 1, c->V.p, ld, c->w.p, c->part.p, nblk, s);
            kr_reduce(c->part.p, nblk, j + 2, c->hcol.p, s);
            kr_update(N, j + 1, c->V.p, ld, c->hcol.p, c->w.p, c->part2.p, nblk, s);
            const double *h2 = nullptr;
            if (c->opt.reorth) {
                kr_mdot(N, j + 1, c->V.p, ld, c->w.p, c->part.p, nblk, s);
                kr_reduce(c->part.p, nblk, j + 2, c->hcol2.p, s);
                kr_update(N, j + 1, c->V.p, ld, c->hcol2.p, c->w.p, c->part2.p, nblk, s);
                h2 = c->hcol2.p;
            }
            kr_arnoldi_finish2(j, m, c->Hm.p, c->cs.p, c->sn.p, c->g.p, c->hcol.p, h2, c->part2.p, nblk, c->scal.p,
                               c->hinfo.p, s);
            kr_scale(N, c->w.p, c->scal.p, c->V.p + (size_t)(j + 1) * ld, s);
            c->mark(5);
            read_bytes(c->hinfo_host, c->hinfo.p, 3 * sizeof(double), s);
            if (c->opt.timing) {
                CPTR_HIP(hipEventSynchronize(c->tev[5]));
                for (int q = 0; q < 5; ++q) {
                    float ms = 0.f;
                    CPTR_HIP(hipEventElapsedTime(&ms, c->tev[q], c->tev[q + 1]));
                    c->tacc[q] += ms;
                }
                c->tsteps++;
            }
            ++its;
            k = j + 1;
            const double gres = c->hinfo_host[0], hj1 = c->hinfo_host[1], wn0 = c->hinfo_host[2];
            if (!std::isfinite(gres) || !std::isfinite(hj1)) {
                set_error("non-finite value in the Arnoldi process");
                return CPTR_E_NONFINITE;
            }
            c->history.push_back(gres / bnorm);
            if (hj1 <= 1e-14 * wn0) { breakdown = true; break; }
            if (gres <= target || its >= c->opt.max_iters) break;
        }
        kr_solve_upper(k, m, c->Hm.p, c->g.p, c->y.p, s);
        kr_combine<double>(N, k, c->Z.p, ld, c->y.p, c->x.p, s);
        launch_bsr_residual(c->n, c->b, c->rp.p, c->ci.p, c->abar.p, c->x.p, c->rhsbar.p, c->r.p, s);
        const double rn = device_norm(c, c->r.p, N);
        if (!std::isfinite(rn)) {
            set_error("non-finite residual");
            return CPTR_E_NONFINITE;
        }
        true_rel = rn / bnorm;
        bool ok = true_rel <= c->opt.rtol;
        if (unscaled) {
            const double ru = unscaled_norm(c, c->r.p) / bnorm0;
            if (!std::isfinite(ru)) {
                set_error("non-finite residual");
                return CPTR_E_NONFINITE;
            }
            if (ru > c->opt.rtol) {
                ok = false;
                target = std::min(target, rn * (c->opt.rtol / ru) * 0.5);
            }
        }
        if (ok) { converged = true; break; }
        if (its >= c->opt.max_iters) break;
        if (breakdown && rn == 0.0) break;
        ++restarts;
    }
    res->iterations = its;
    res->restarts = restarts;
    res->converged = converged ? 1 : 0;
    res->rel_res_scaled = true_rel;
    res->timed_steps = c->tsteps;
    res->t_stage1_ms = c->tacc[0];
    res->t_stage2_ms = c->tacc[1];
    res->t_last_ms = c->tacc[2];
    res->t_spmv_ms = c->tacc[3];
    res->t_arnoldi_ms = c->tacc[4];
    return converged ? CPTR_OK : CPTR_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
#define CPTR_API_BEGIN try {
#define CPTR_API_END                                                   \
    }                                                                  \
    catch (const Error &e) {                                           \
        set_error(e.what());                                           \
        return e.status;                                               \
    }                                                                  \
    catch (const std::exception &e) {                                  \
        set_error(e.what());                                           \
        return CPTR_E_HIP;                                             \
    }

extern "C" {

const char *cptr_last_error(void) { return g_last_error.c_str(); }

cptr_status cptr_default_options(cptr_options *o) {
    if (!o) { set_error("null options"); return CPTR_E_ARG; }
    std::memset(o, 0, sizeof(*o));
    o->variant = CPTR_VARIANT_CPTR3;
    o->stage_order = CPTR_T_THEN_P;
    o->last_stage = CPTR_LAST_BILU0;
    o->krylov = CPTR_GMRES;
    o->restart = 30;
    o->max_iters = 1000;
    o->rtol = 1e-8;
    o->precond_precision = CPTR_FP64;
    o->reorth = 0;
    o->amg_theta = 0.25;
    o->amg_max_coarse = 1000;
    o->amg_max_levels = 25;
    o->amg_pmax = 4;
    o->smoother = CPTR_SMOOTH_JACOBI;
    o->pre_sweeps = 1;
    o->post_sweeps = 1;
    o->jacobi_omega = 2.0 / 3.0;
    o->pmis_seed = 0;
    o->ilu_tile_x = 32;
    o->ilu_tile_y = 8;
    o->t_interp = CPTR_INTERP_CLASSICAL;
    o->reuse_rho_max = 0.3;
    o->timing = 0;
    o->setup_kernels = 0;
    o->exact_subsolves = 0;
    o->cheb_degree = 2;
    o->stop_unscaled = 0;
    o->judge_cycles = 4;
    return CPTR_OK;
}

cptr_status cptr_create(cptr_ctx **out, int32_t dev, void *stream, const cptr_options *opt) {
    CPTR_API_BEGIN
    if (!out) throw Error(CPTR_E_ARG, "null context pointer");
    *out = nullptr;
    int ndev = 0;
    CPTR_HIP(hipGetDeviceCount(&ndev));
    if (dev < 0 || dev >= ndev) throw Error(CPTR_E_ARG, "invalid HIP device");
    CPTR_HIP(hipSetDevice(dev));
    StreamScope scope((hipStream_t)stream);
    auto c = std::make_unique<cptr_ctx>();
    c->device = dev;
    c->stream = (hipStream_t)stream;
    if (opt) c->opt = *opt;
    else cptr_default_options(&c->opt);
    validate_options(c->opt);
    c->flag.alloc(4);
    fill_int(c->flag.p, 0, 1, c->stream);
    CPTR_HIP(hipEventCreate(&c->ev0));
    CPTR_HIP(hipEventCreate(&c->ev1));
    for (auto &e : c->tev) CPTR_HIP(hipEventCreate(&e));
    CPTR_HIP(hipEventCreateWithFlags(&c->ev_dec, hipEventDisableTiming));
    for (int k = 0; k < 3; ++k) {
        CPTR_HIP(hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking));   // default priority
        CPTR_HIP(hipEventCreateWithFlags(&c->ev_side[k], hipEventDisableTiming));
    }
    CPTR_HIP(hipStreamCreateWithFlags(&c->side_trial, hipStreamNonBlocking));   // default priority
    CPTR_HIP(hipStreamSynchronize(c->stream));
    *out = c.release();
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_destroy(cptr_ctx *c) {
    CPTR_API_BEGIN
    if (!c) return CPTR_OK;
    CPTR_HIP(hipSetDevice(c->device));
    StreamScope scope(c->stream);
    CPTR_HIP(hipStreamSynchronize(c->stream));
    hipStream_t s = c->stream;
    delete c;
    pool_trim(s);
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_setup(cptr_ctx *c, int32_t n, int32_t b, int32_t nnzb, const int32_t *d_rp, const int32_t *d_ci,
                       const double *d_vals, int32_t p_index, int32_t T_index, int32_t nx, int32_t ny) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    if (!c) throw Error(CPTR_E_ARG, "null context");
    CPTR_HIP(hipSetDevice(c->device));
    if (n <= 0 || nnzb < n || b < 2 || b > 8) throw Error(CPTR_E_ARG, "need n > 0, nnzb >= n, 2 <= b <= 8");
    if (!d_rp || !d_ci || !d_vals) throw Error(CPTR_E_ARG, "null matrix pointer");
    if (p_index < 0 || p_index >= b || T_index < 0 || T_index >= b || p_index == T_index)
        throw Error(CPTR_E_ARG, "invalid pressure / temperature index");
    const bool grid = (nx > 0 && ny > 0);
    if (grid && (long)nx * ny != n) throw Error(CPTR_E_ARG, "nx * ny must equal n_cells");
    if (c->opt.last_stage == CPTR_LAST_BILU0 && !grid)
        throw Error(CPTR_E_ARG, "BILU(0) needs the grid shape (nx, ny); use block Jacobi otherwise");
    hipStream_t s = c->stream;
    c->ready = false;
    CPTR_HIP(hipEventRecord(c->ev0, s));
    c->n = n; c->b = b; c->nnzb = nnzb; c->ip = p_index; c->it = T_index; c->nx = nx; c->ny = ny;
    c->rp.alloc((size_t)n + 1);
    c->ci.alloc(nnzb);
    CPTR_HIP(hipMemcpyAsync(c->rp.p, d_rp, sizeof(int) * (n + 1), hipMemcpyDeviceToDevice, s));
    CPTR_HIP(hipMemcpyAsync(c->ci.p, d_ci, sizeof(int) * nnzb, hipMemcpyDeviceToDevice, s));
    int last = read_scalar(c->rp.p + n, s);
    int first = read_scalar(c->rp.p, s);
    if (first != 0 || last != nnzb) throw Error(CPTR_E_ARG, "row_ptr[0] must be 0 and row_ptr[n] = nnzb");
    check_pattern(n, c->rp.p, c->ci.p, c->flag.p, s);
    c->tpos.alloc(nnzb);
    transpose_index(n, c->rp.p, c->ci.p, c->tpos.p, c->flag.p, s);
    if (grid && nx >= 2) check_grid5(n, nx, c->rp.p, c->ci.p, c->flag.p, s);
    int f = read_flag_and_clear(c);
    c->ell5 = grid && nx >= 2 && !(f & 512);
    if (f & 1) throw Error(CPTR_E_ARG, "block column index out of range");
    if (f & 2) throw Error(CPTR_E_ARG, "block columns must ascend within each row");
    if (f & 4) throw Error(CPTR_E_ARG, "missing diagonal block");
    if (f & 8) throw Error(CPTR_E_ARG, "block pattern is not structurally symmetric");
    c->use_tiles = (c->opt.last_stage == CPTR_LAST_BILU0);
    if (c->use_tiles) {
        tiles_build(c->ts, n, nx, ny, c->opt.ilu_tile_x, c->opt.ilu_tile_y, c->rp.p, c->ci.p, c->flag.p, s);
        if (read_flag_and_clear(c) & 128)
            throw Error(CPTR_E_ARG, "BILU(0) tile order needs a 5-point grid pattern; use block Jacobi");
    }
    for (auto &h : c->H) h.built = false;
    c->rho[0] = c->rho[1] = -1.0;
    c->reused = 0;
    c->skip_left[0] = c->skip_left[1] = 0;
    c->backoff[0] = c->backoff[1] = 1;
    do_setup_values(c, d_vals, false);
    alloc_krylov(c);
    CPTR_HIP(hipEventRecord(c->ev1, s));
    CPTR_HIP(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    CPTR_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_setup_ms = ms;
    c->ready = true;
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_update_values(cptr_ctx *c, const double *d_vals) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    if (!c || !c->ready) throw Error(CPTR_E_STATE, "update_values before setup");
    CPTR_HIP(hipSetDevice(c->device));
    if (!d_vals) throw Error(CPTR_E_ARG, "null matrix pointer");
    CPTR_HIP(hipEventRecord(c->ev0, c->stream));
    c->ready = false;
    do_setup_values(c, d_vals, c->opt.reuse_rho_max > 0.0);
    c->ready = true;
    CPTR_HIP(hipEventRecord(c->ev1, c->stream));
    CPTR_HIP(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    CPTR_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_setup_ms = ms;
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_solve(cptr_ctx *c, const double *d_rhs, double *d_x, cptr_result *out) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    if (!c || !c->ready) throw Error(CPTR_E_STATE, "solve before setup");
    if (!d_rhs || !d_x) throw Error(CPTR_E_ARG, "null vector");
    CPTR_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    cptr_result res{};
    CPTR_HIP(hipEventRecord(c->ev0, s));
    const int N = c->n * c->b;
    count_nonfinite(d_rhs, (size_t)N, c->flag.p, s);
    if (read_flag_and_clear(c) & 16) throw Error(CPTR_E_NONFINITE, "non-finite right-hand side");
    if (c->opt.variant == CPTR_VARIANT_LAST_ONLY)
        CPTR_HIP(hipMemcpyAsync(c->rhsbar.p, d_rhs, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    else
        launch_scale_rhs(c->opt.variant, c->n, c->b, d_rhs, c->ip, c->it, c->wp.p, c->wt.p, c->beta.p, c->rhsbar.p, s);
    const double bn = device_norm(c, d_rhs, N);
    cptr_status st = run_gmres(c, &res, bn);
    if (st < 0) return st;
    CPTR_HIP(hipMemcpyAsync(d_x, c->x.p, sizeof(double) * N, hipMemcpyDeviceToDevice, s));
    const double rn = unscaled_norm(c, c->r.p);
    res.rel_res_unscaled = (bn > 0) ? rn / bn : 0.0;
    CPTR_HIP(hipEventRecord(c->ev1, s));
    CPTR_HIP(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    CPTR_HIP(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    res.solve_ms = ms;
    res.setup_ms = c->last_setup_ms;
    res.levels_T = (int)c->H[0].L.size();
    res.levels_P = (int)c->H[1].L.size();
    res.rho_T = c->rho[0];
    res.rho_P = c->rho[1];
    res.reused = c->reused;
    res.used_learned = c->used_learned;
    res.rho_T_classical = c->rho_cls;
    res.rho_T_learned = c->rho_lrn;
    res.t_setup_scale_ms = c->tph[0];
    res.t_setup_amgT_ms = c->tph[1];
    res.t_setup_amgP_ms = c->tph[2];
    res.t_setup_values_ms = c->tph[3];
    if (out) *out = res;
    return st;
    CPTR_API_END
}

cptr_status cptr_residual_history(const cptr_ctx *c, double *buf, int32_t cap, int32_t *len) {
    CPTR_API_BEGIN
    if (!c || !len) throw Error(CPTR_E_ARG, "null argument");
    int k = (int)c->history.size();
    *len = k;
    if (buf)
        for (int i = 0; i < k && i < cap; ++i) buf[i] = c->history[i];
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_decouple(int32_t variant, int32_t n, int32_t b, const int32_t *d_rp, const int32_t *d_ci,
                          const double *d_vals, const double *d_rhs, int32_t ip, int32_t it, double *d_abar,
                          double *d_rhsbar, void *stream) {
    CPTR_API_BEGIN
    StreamScope scope((hipStream_t)stream);
    if (variant != CPTR_VARIANT_CPTR3 && variant != CPTR_VARIANT_CPR && variant != CPTR_VARIANT_CPTR)
        throw Error(CPTR_E_ARG, "variant");
    if (n <= 0 || b < 2 || b > 8) throw Error(CPTR_E_ARG, "sizes");
    hipStream_t s = (hipStream_t)stream;
    DBuf<double> wp, wt, beta;
    DBuf<int> err;
    wp.alloc((size_t)n * b);
    wt.alloc((size_t)n * b);
    beta.alloc(n);
    err.alloc(1);
    fill_int(err.p, 0x7fffffff, 1, s);
    launch_decouple(variant, n, b, d_rp, d_ci, d_vals, ip, it, d_abar, wp.p, wt.p, beta.p, err.p, s);
    if (d_rhs && d_rhsbar) launch_scale_rhs(variant, n, b, d_rhs, ip, it, wp.p, wt.p, beta.p, d_rhsbar, s);
    int bad = read_scalar(err.p, s);
    if (bad != 0x7fffffff) throw Error(CPTR_E_SINGULAR_BLOCK, "singular decoupling block in cell " + std::to_string(bad));
    return CPTR_OK;
    CPTR_API_END
}

// The decoupling without allocation (cptr_decouple_noalloc): the weights,
// beta and the singular-cell word live in this file-scope device array, one
// copy per GPU, whose address is looked up once per device.  Calls that
// overlap on one GPU share it and race.
static __device__ __align__(256) unsigned char scratch[CPTR_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64] = {};

static unsigned char *scratch_on_current_device() {
    int dev = 0;
    CPTR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) throw Error(CPTR_E_ARG, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        CPTR_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw Error(CPTR_E_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    return (unsigned char *)g_scratch_ptr[dev];
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

cptr_status cptr_decouple_noalloc(int32_t variant, int32_t n, int32_t b, const int32_t *d_rp, const int32_t *d_ci,
                                  const double *d_vals, const double *d_rhs, int32_t ip, int32_t it, double *d_abar,
                                  double *d_rhsbar, void *stream) {
    CPTR_API_BEGIN
    if (variant != CPTR_VARIANT_CPTR3 && variant != CPTR_VARIANT_CPR && variant != CPTR_VARIANT_CPTR)
        throw Error(CPTR_E_ARG, "variant");
    if (n <= 0 || b < 2 || b > 8) throw Error(CPTR_E_ARG, "sizes");
    if (!d_rp || !d_ci || !d_vals || !d_abar) throw Error(CPTR_E_ARG, "null pointer");
    if (ip < 0 || ip >= b || it < 0 || it >= b || ip == it)
        throw Error(CPTR_E_ARG, "invalid pressure / temperature index");
    // layout: the singular-cell word, w_P and w_T (n*b each), beta (n)
    const size_t o_wp = 256;
    const size_t o_wt = o_wp + align256((size_t)n * b * sizeof(double));
    const size_t o_beta = o_wt + align256((size_t)n * b * sizeof(double));
    const size_t need = o_beta + align256((size_t)n * sizeof(double));
    if (need > (size_t)CPTR_NOALLOC_SCRATCH_BYTES)
        throw Error(CPTR_E_ARG, "decouple_noalloc: " + std::to_string(n) + " cells of block size " +
                                    std::to_string(b) + " need " + std::to_string(need) +
                                    " bytes of scratch, above the limit of " +
                                    std::to_string((size_t)CPTR_NOALLOC_SCRATCH_BYTES));
    hipStream_t s = (hipStream_t)stream;
    unsigned char *base = scratch_on_current_device();
    int *err = (int *)base;
    double *wp = (double *)(base + o_wp), *wt = (double *)(base + o_wt), *beta = (double *)(base + o_beta);
    fill_int(err, 0x7fffffff, 1, s);
    launch_decouple(variant, n, b, d_rp, d_ci, d_vals, ip, it, d_abar, wp, wt, beta, err, s);
    if (d_rhs && d_rhsbar) launch_scale_rhs(variant, n, b, d_rhs, ip, it, wp, wt, beta, d_rhsbar, s);
    int bad = 0;
    CPTR_HIP(hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, s));
    CPTR_HIP(hipStreamSynchronize(s));
    if (bad != 0x7fffffff) throw Error(CPTR_E_SINGULAR_BLOCK, "singular decoupling block in cell " + std::to_string(bad));
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_stream_read(const double *d_x, uint64_t n, double *d_part, int32_t *blocks, void *stream) {
    CPTR_API_BEGIN
    if (!blocks) throw Error(CPTR_E_ARG, "null blocks");
    *blocks = stream_read_blocks((size_t)n);
    if (!d_x && !d_part) return CPTR_OK;       // size query
    if (!d_x || !d_part) throw Error(CPTR_E_ARG, "null pointer");
    if ((uintptr_t)d_x & 15) throw Error(CPTR_E_ARG, "d_x must be 16-byte aligned");
    if (n == 0) return CPTR_OK;
    launch_stream_read((size_t)n, d_x, d_part, (hipStream_t)stream);
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_bsr_spmv(int32_t n, int32_t b, const int32_t *d_rp, const int32_t *d_ci, const double *d_vals,
                          const double *d_x, double *d_y, void *stream) {
    CPTR_API_BEGIN
    if (n < 0 || b < 1 || b > 8) throw Error(CPTR_E_ARG, "sizes");
    if (b == 8 && (((uintptr_t)d_vals | (uintptr_t)d_x) & 15))
        throw Error(CPTR_E_ARG, "block size 8 needs 16-byte aligned values and x");
    launch_bsr_spmv(n, b, d_rp, d_ci, d_vals, d_x, d_y, (hipStream_t)stream);
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_condense(int32_t n, int32_t n1, int32_t n2, int32_t nnzb, const int32_t *d_rp, const int32_t *d_ci,
                          const double *d_J11, const double *d_J12, const double *d_J21, const double *d_J22,
                          const double *d_r1, const double *d_r2, double *d_A, double *d_b, double *d_Q,
                          double *d_q, void *stream) {
    CPTR_API_BEGIN
    if (n < 0 || nnzb < n || n1 < 1 || n1 > 8 || n2 < 0 || n2 > 8)
        throw Error(CPTR_E_ARG, "sizes: n1 must be 1..8, n2 0..8, nnzb >= n_cells");
    if (n == 0) return CPTR_OK;
    if (!d_rp || !d_ci || !d_J11 || !d_r1 || !d_A || !d_b) throw Error(CPTR_E_ARG, "null pointer");
    if (n2 > 0 && (!d_J12 || !d_J21 || !d_J22 || !d_r2 || !d_Q || !d_q)) throw Error(CPTR_E_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    StreamScope scope(s);
    DBuf<int> flag;
    flag.alloc(1);
    fill_int(flag.p, 0x7fffffff, 1, s);
    launch_condense_cells(n, n1, n2, d_J21, d_J22, d_r2, d_Q, d_q, flag.p, s);
    const int bad = read_scalar(flag.p, s);
    if (bad != 0x7fffffff)
        throw Error(CPTR_E_SINGULAR_BLOCK, "singular secondary block J22 in cell " + std::to_string(bad));
    launch_condense_blocks(n, n1, n2, d_rp, d_ci, d_J11, d_J12, d_Q, d_q, d_r1, d_A, d_b, s);
    CPTR_HIP(hipStreamSynchronize(s));
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_condense_wells(int32_t n, int32_t n1, int32_t nnzb, const int32_t *d_rp, const int32_t *d_ci,
                                int32_t n_wells, int32_t nw, const int32_t *d_well_cell, const double *d_J1w,
                                const double *d_Jw1, const double *d_Jww, const double *d_rw, double *d_A, double *d_b,
                                double *d_Qw, double *d_qw, void *stream) {
    CPTR_API_BEGIN
    if (n < 0 || nnzb < n || n1 < 1 || n1 > 8 || nw < 1 || nw > 8 || n_wells < 0)
        throw Error(CPTR_E_ARG, "sizes: n1 must be 1..8, nw 1..8, n_wells >= 0, nnzb >= n_cells");
    if (n_wells == 0) return CPTR_OK;
    if (n == 0) throw Error(CPTR_E_ARG, "wells need cells");
    if (!d_rp || !d_ci || !d_well_cell || !d_J1w || !d_Jw1 || !d_Jww || !d_rw || !d_A || !d_b || !d_Qw || !d_qw)
        throw Error(CPTR_E_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    StreamScope scope(s);
    std::vector<int> cells((size_t)n_wells);
    CPTR_HIP(hipMemcpyAsync(cells.data(), d_well_cell, sizeof(int) * n_wells, hipMemcpyDeviceToHost, s));
    CPTR_HIP(hipStreamSynchronize(s));
    for (int w = 0; w < n_wells; ++w)
        if (cells[w] < 0 || cells[w] >= n)
            throw Error(CPTR_E_ARG, "well " + std::to_string(w) + " perforates cell " + std::to_string(cells[w]) +
                                        ", outside 0.." + std::to_string(n - 1));
    DBuf<int> flag;
    flag.alloc(2);
    fill_int(flag.p, 0x7fffffff, 2, s);
    launch_condense_wells(n_wells, n1, nw, d_rp, d_ci, d_well_cell, d_J1w, d_Jw1, d_Jww, d_rw, d_A, d_b, d_Qw, d_qw,
                          flag.p, s);
    int bad[2];
    read_bytes(bad, flag.p, sizeof(bad), s);
    if (bad[1] != 0x7fffffff)
        throw Error(CPTR_E_ARG, "the cell of well " + std::to_string(bad[1]) + " has no diagonal block");
    if (bad[0] != 0x7fffffff)
        throw Error(CPTR_E_SINGULAR_BLOCK, "singular well block Jww in well " + std::to_string(bad[0]));
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_recover_wells(int32_t n_wells, int32_t n1, int32_t nw, const int32_t *d_well_cell,
                               const double *d_Qw, const double *d_qw, const double *d_delta1, double *d_deltaw,
                               void *stream) {
    CPTR_API_BEGIN
    if (n_wells < 0 || n1 < 1 || n1 > 8 || nw < 1 || nw > 8) throw Error(CPTR_E_ARG, "sizes: n1 and nw must be 1..8");
    if (n_wells == 0) return CPTR_OK;
    if (!d_well_cell || !d_Qw || !d_qw || !d_delta1 || !d_deltaw) throw Error(CPTR_E_ARG, "null pointer");
    launch_recover_wells(n_wells, n1, nw, d_well_cell, d_Qw, d_qw, d_delta1, d_deltaw, (hipStream_t)stream);
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_recover_secondary(int32_t n, int32_t n1, int32_t n2, const double *d_Q, const double *d_q,
                                   const double *d_d1, double *d_d2, void *stream) {
    CPTR_API_BEGIN
    if (n < 0 || n1 < 1 || n1 > 8 || n2 < 0 || n2 > 8) throw Error(CPTR_E_ARG, "sizes: n1 must be 1..8, n2 0..8");
    if (n == 0 || n2 == 0) return CPTR_OK;
    if (!d_Q || !d_q || !d_d1 || !d_d2) throw Error(CPTR_E_ARG, "null pointer");
    launch_condense_recover(n, n1, n2, d_Q, d_q, d_d1, d_d2, (hipStream_t)stream);
    return CPTR_OK;
    CPTR_API_END
}

static Hierarchy &pick(const cptr_ctx *c, int which) {
    if (!c || !c->ready) throw Error(CPTR_E_STATE, "context not set up");
    if (which < 0 || which > 1) throw Error(CPTR_E_ARG, "which must be 0 (T) or 1 (P)");
    Hierarchy &h = const_cast<cptr_ctx *>(c)->H[which];
    if (!h.built) throw Error(CPTR_E_STATE, "hierarchy not built for this variant");
    return h;
}

cptr_status cptr_amg_levels(const cptr_ctx *c, int32_t which, int32_t *levels) {
    CPTR_API_BEGIN
    *levels = (int)pick(c, which).L.size();
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_amg_level_info(const cptr_ctx *c, int32_t which, int32_t level, int32_t *nrows, int32_t *nnz,
                                int32_t *p_nnz) {
    CPTR_API_BEGIN
    Hierarchy &h = pick(c, which);
    if (level < 0 || level >= (int)h.L.size()) throw Error(CPTR_E_ARG, "level out of range");
    const Level &L = h.L[level];
    if (nrows) *nrows = L.A.n;
    if (nnz) *nnz = L.A.nnz;
    if (p_nnz) *p_nnz = (level + 1 < (int)h.L.size()) ? L.P.nnz : 0;
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_amg_level_copy(const cptr_ctx *c, int32_t which, int32_t level, int32_t *h_rp, int32_t *h_ci,
                                double *h_v, int32_t *h_cf, int32_t *h_prp, int32_t *h_pci, double *h_pv) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    Hierarchy &h = pick(c, which);
    if (level < 0 || level >= (int)h.L.size()) throw Error(CPTR_E_ARG, "level out of range");
    CPTR_HIP(hipSetDevice(c->device));
    const Level &L = h.L[level];
    hipStream_t s = c->stream;
    if (h_rp) CPTR_HIP(hipMemcpyAsync(h_rp, L.A.rp, sizeof(int) * (L.A.n + 1), hipMemcpyDeviceToHost, s));
    if (h_ci) CPTR_HIP(hipMemcpyAsync(h_ci, L.A.ci, sizeof(int) * L.A.nnz, hipMemcpyDeviceToHost, s));
    if (h_v) CPTR_HIP(hipMemcpyAsync(h_v, L.A.v.p, sizeof(double) * L.A.nnz, hipMemcpyDeviceToHost, s));
    const bool has_p = level + 1 < (int)h.L.size();
    if (h_cf && has_p) CPTR_HIP(hipMemcpyAsync(h_cf, L.cf.p, sizeof(int) * L.A.n, hipMemcpyDeviceToHost, s));
    if (has_p) {
        if (h_prp) CPTR_HIP(hipMemcpyAsync(h_prp, L.P.rp, sizeof(int) * (L.P.n + 1), hipMemcpyDeviceToHost, s));
        if (h_pci) CPTR_HIP(hipMemcpyAsync(h_pci, L.P.ci, sizeof(int) * L.P.nnz, hipMemcpyDeviceToHost, s));
        if (h_pv) CPTR_HIP(hipMemcpyAsync(h_pv, L.P.v.p, sizeof(double) * L.P.nnz, hipMemcpyDeviceToHost, s));
    }
    CPTR_HIP(hipStreamSynchronize(s));
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_amg_vcycle(cptr_ctx *c, int32_t which, const double *d_b, double *d_x) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    Hierarchy &h = pick(c, which);
    CPTR_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int n = h.L[0].A.n;
    CPTR_HIP(hipMemcpyAsync(h.L[0].b.p, d_b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    double *x = vcycle<double>(c, h, 0, s);
    CPTR_HIP(hipMemcpyAsync(d_x, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    CPTR_HIP(hipStreamSynchronize(s));
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_amg_conv_factor(cptr_ctx *c, int32_t which, int32_t cycles, uint64_t seed, double *rho) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    Hierarchy &h = pick(c, which);
    if (cycles < 1 || cycles > 1000) throw Error(CPTR_E_ARG, "cycles must be 1..1000");
    if (!rho) throw Error(CPTR_E_ARG, "null output");
    CPTR_HIP(hipSetDevice(c->device));
    *rho = conv_factor(c, h, cycles, seed, c->stream);
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_precond_apply(cptr_ctx *c, const double *d_r, double *d_y) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    if (!c || !c->ready) throw Error(CPTR_E_STATE, "context not set up");
    CPTR_HIP(hipSetDevice(c->device));
    precond(c, d_r, d_y);
    CPTR_HIP(hipStreamSynchronize(c->stream));
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_get_scaled(const cptr_ctx *c, double *d_abar, double *d_rhsbar, const double *d_rhs) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    if (!c || !c->ready) throw Error(CPTR_E_STATE, "context not set up");
    CPTR_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    if (d_abar)
        CPTR_HIP(hipMemcpyAsync(d_abar, c->abar.p, sizeof(double) * c->nnzb * c->b * c->b, hipMemcpyDeviceToDevice, s));
    if (d_rhsbar && d_rhs) {
        if (c->opt.variant == CPTR_VARIANT_LAST_ONLY)
            CPTR_HIP(hipMemcpyAsync(d_rhsbar, d_rhs, sizeof(double) * c->n * c->b, hipMemcpyDeviceToDevice, s));
        else
            launch_scale_rhs(c->opt.variant, c->n, c->b, d_rhs, c->ip, c->it, c->wp.p, c->wt.p, c->beta.p, d_rhsbar, s);
    }
    CPTR_HIP(hipStreamSynchronize(s));
    return CPTR_OK;
    CPTR_API_END
}

struct cptr_mlp {
    int device = 0;
    DBuf<float> p, m, v, g;
    int t = 0;
};

static Level &train_level(cptr_ctx *c) {
    if (!c || !c->ready) throw Error(CPTR_E_STATE, "context not set up");
    if (!c->H[0].built || c->H[0].L.size() < 2)
        throw Error(CPTR_E_STATE, "the temperature hierarchy has a single level (no interpolation)");
    if (c->used_learned) throw Error(CPTR_E_STATE, "the temperature interpolation is the learned one, not classical");
    if (c->opt.amg_pmax < 1 || c->opt.amg_pmax > 16)
        throw Error(CPTR_E_ARG, "the learned interpolation needs amg_pmax in 1..16 (edges per row)");
    return c->H[0].L[0];
}

cptr_status cptr_load_mlp(cptr_ctx *c, const float *host_params) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    if (!c) throw Error(CPTR_E_ARG, "null context");
    CPTR_HIP(hipSetDevice(c->device));
    if (!host_params) {
        c->have_mlp = false;
        return CPTR_OK;
    }
    c->mlp.alloc(MLP_NPARAMS);
    CPTR_HIP(hipMemcpyAsync(c->mlp.p, host_params, sizeof(float) * MLP_NPARAMS, hipMemcpyHostToDevice, c->stream));
    CPTR_HIP(hipStreamSynchronize(c->stream));
    c->have_mlp = true;
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_mlp_create(cptr_mlp **out, int32_t dev, const float *host_params) {
    CPTR_API_BEGIN
    if (!out || !host_params) throw Error(CPTR_E_ARG, "null argument");
    *out = nullptr;
    int ndev = 0;
    CPTR_HIP(hipGetDeviceCount(&ndev));
    if (dev < 0 || dev >= ndev) throw Error(CPTR_E_ARG, "invalid HIP device");
    CPTR_HIP(hipSetDevice(dev));
    StreamScope scope(nullptr);
    auto m = std::make_unique<cptr_mlp>();
    m->device = dev;
    m->p.alloc(MLP_NPARAMS);
    m->m.alloc(MLP_NPARAMS);
    m->v.alloc(MLP_NPARAMS);
    m->g.alloc(MLP_NPARAMS);
    CPTR_HIP(hipMemcpy(m->p.p, host_params, sizeof(float) * MLP_NPARAMS, hipMemcpyHostToDevice));
    CPTR_HIP(hipMemset(m->m.p, 0, sizeof(float) * MLP_NPARAMS));
    CPTR_HIP(hipMemset(m->v.p, 0, sizeof(float) * MLP_NPARAMS));
    CPTR_HIP(hipMemset(m->g.p, 0, sizeof(float) * MLP_NPARAMS));
    *out = m.release();
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_mlp_get(const cptr_mlp *m, float *host_params, float *host_grad) {
    CPTR_API_BEGIN
    if (!m) throw Error(CPTR_E_ARG, "null network");
    CPTR_HIP(hipSetDevice(m->device));
    CPTR_HIP(hipDeviceSynchronize());
    if (host_params)
        CPTR_HIP(hipMemcpy(host_params, m->p.p, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToHost));
    if (host_grad) CPTR_HIP(hipMemcpy(host_grad, m->g.p, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToHost));
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_mlp_destroy(cptr_mlp *m) {
    CPTR_API_BEGIN
    if (!m) return CPTR_OK;
    CPTR_HIP(hipSetDevice(m->device));
    CPTR_HIP(hipDeviceSynchronize());
    StreamScope scope(nullptr);
    delete m;
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_mlp_train_step(cptr_mlp *m, cptr_ctx *c, int32_t K, uint64_t seed, double lr, double *loss) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    if (!m) throw Error(CPTR_E_ARG, "null network");
    if (K < 1 || K > 16) throw Error(CPTR_E_ARG, "n_vectors must be 1..16");
    if (!(lr > 0.0)) throw Error(CPTR_E_ARG, "learning rate must be positive");
    Level &L = train_level(c);
    if (m->device != c->device) throw Error(CPTR_E_ARG, "network and context on different devices");
    CPTR_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    const int n = L.A.n;
    EdgeSet es;
    edges_build(s, L, es);
    if (es.E == 0 || es.nf == 0) throw Error(CPTR_E_STATE, "no F-row edges to train on");
    // smooth vectors
    DBuf<double> Ev, tmp;
    Ev.alloc((size_t)K * n);
    tmp.alloc(n);
    vc_hash_uniform(K * n, seed, Ev.p, s);
    for (int k = 0; k < K; ++k) {
        double *e = Ev.p + (size_t)k * n;
        for (int sw = 0; sw < 20; sw += 2) {
            ln_jacobi_zero(n, L.A.rp, L.A.ci, L.A.v.p, 2.0 / 3.0, e, tmp.p, s);
            ln_jacobi_zero(n, L.A.rp, L.A.ci, L.A.v.p, 2.0 / 3.0, tmp.p, e, s);
        }
    }
    // forward, loss and dL/do, backward, reduction, Adam
    DBuf<float> o, dout, part;
    DBuf<double> lrow, lsum;
    o.alloc(es.E);
    dout.alloc(es.E);
    lrow.alloc(es.nf);
    lsum.alloc(1);
    ln_mlp_forward(es.E, es.X.p, m->p.p, o.p, s);
    ln_interp_loss(es.nf, n, K, es.frows.p, es.estart.p, L.P.rp, L.P.ci, L.P.v.p, es.fine_of.p, Ev.p, o.p, lrow.p,
                   dout.p, s);
    kr_reduce(lrow.p, es.nf, 1, lsum.p, s);
    const int nw = ln_mlp_waves(es.E);
    part.alloc((size_t)nw * MLP_NPARAMS);
    ln_mlp_backward(es.E, es.X.p, m->p.p, dout.p, part.p, s);
    ln_grad_reduce(nw, part.p, m->g.p, s);
    m->t += 1;
    ln_adam(m->p.p, m->m.p, m->v.p, m->g.p, lr, 0.9, 0.999, 1e-8, m->t, s);
    const double tot = read_scalar(lsum.p, s);
    if (loss) *loss = tot / es.nf;
    return CPTR_OK;
    CPTR_API_END
}

cptr_status cptr_mlp_edges(const cptr_mlp *m, cptr_ctx *c, float *host_X, float *host_o, int32_t cap,
                           int32_t *n_edges) {
    CPTR_API_BEGIN
    StreamScope scope(c ? c->stream : nullptr);
    if (!n_edges) throw Error(CPTR_E_ARG, "null count");
    Level &L = train_level(c);
    CPTR_HIP(hipSetDevice(c->device));
    hipStream_t s = c->stream;
    EdgeSet es;
    edges_build(s, L, es);
    *n_edges = es.E;
    const int k = std::min(es.E, (int)std::max(cap, 0));
    if (host_X && k > 0)
        CPTR_HIP(hipMemcpyAsync(host_X, es.X.p, sizeof(float) * MLP_NF * k, hipMemcpyDeviceToHost, s));
    if (host_o && m && k > 0) {
        DBuf<float> o;
        o.alloc(es.E);
        ln_mlp_forward(es.E, es.X.p, m->p.p, o.p, s);
        CPTR_HIP(hipMemcpyAsync(host_o, o.p, sizeof(float) * k, hipMemcpyDeviceToHost, s));
        CPTR_HIP(hipStreamSynchronize(s));
    }
    CPTR_HIP(hipStreamSynchronize(s));
    return CPTR_OK;
    CPTR_API_END
}

}  // extern "C"
