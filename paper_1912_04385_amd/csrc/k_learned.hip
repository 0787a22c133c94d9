// Learned fine-level interpolation of the temperature AMG stage (an
// extension of amg(C_TT), Eq. CPTR3M1): a 16 -> 64 -> 64 -> 1 edge-MLP with
// BF16 weights corrects the classical extended+i weights of every F row,
//   w_e = w0_e (1 + tanh(o_e) / 2), rescaled to the classical row sum,
// and is trained on smooth error vectors of the operator itself.
//
// Edges are the entries of the classical interpolation P in F rows, in P's
// storage order.  The network runs on the matrix cores: one wavefront per
// tile of 32 edges, v_mfma_f32_32x32x8_bf16 with FP32 accumulation, the
// layer operands staged through LDS.  Feature, loss and weight arithmetic is
// FP64 (this file is compiled without floating-point contraction).
#include "internal.h"

namespace cptr {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TILE = 32;          // edges per wavefront tile
constexpr int WAVES = 2;          // wavefronts per block
constexpr int THREADS = 64 * WAVES;

// round-to-nearest-even FP32 -> BF16 (inputs are finite)
__device__ inline unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

// parameter blob offsets
constexpr int OW1 = 0, OB1 = OW1 + MLP_NH * MLP_NF, OW2 = OB1 + MLP_NH, OB2 = OW2 + MLP_NH * MLP_NH,
              OW3 = OB2 + MLP_NH, OB3 = OW3 + MLP_NH;

struct Weights {
    unsigned short w1[MLP_NH * MLP_NF];   // [h][f]
    unsigned short w2[MLP_NH * MLP_NH];   // [h2][h1]
    float w3[MLP_NH];                     // BF16 values held in FP32
    float b1[MLP_NH], b2[MLP_NH], b3;
};

struct WaveBuf {
    unsigned short x[TILE * MLP_NF];      // inputs (BF16)
    unsigned short h1[TILE * MLP_NH];     // first hidden layer after ReLU (BF16)
    float h2[TILE * MLP_NH];              // second hidden layer after ReLU (FP32); dz1 in the backward pass
    unsigned short d2[TILE * MLP_NH];     // dz2 (BF16)
    unsigned short d1[TILE * MLP_NH];     // dz1 (BF16)
};

__device__ void load_weights(const float *__restrict__ p, Weights &W) {
    for (int k = threadIdx.x; k < MLP_NH * MLP_NF; k += blockDim.x) W.w1[k] = f2bf(p[OW1 + k]);
    for (int k = threadIdx.x; k < MLP_NH * MLP_NH; k += blockDim.x) W.w2[k] = f2bf(p[OW2 + k]);
    for (int k = threadIdx.x; k < MLP_NH; k += blockDim.x) {
        W.w3[k] = bf2f(f2bf(p[OW3 + k]));
        W.b1[k] = p[OB1 + k];
        W.b2[k] = p[OB2 + k];
    }
    if (threadIdx.x == 0) W.b3 = p[OB3];
}

// stage the features of tile `t` (zeros past the last edge)
__device__ void load_tile(int lane, long t, int E, const float *__restrict__ X, WaveBuf &B) {
    const int le = lane >> 1, f0 = (lane & 1) * 8;
    const long e = t * TILE + le;
    for (int q = 0; q < 8; ++q) B.x[le * MLP_NF + f0 + q] = (e < E) ? f2bf(X[e * MLP_NF + f0 + q]) : 0;
}

// forward pass of one tile: h1 (BF16) and h2 (FP32) into LDS
__device__ void forward_tile(int lane, const Weights &W, WaveBuf &B) {
    const int lr = lane & 31, lk = 4 * (lane >> 5);
    for (int nb = 0; nb < 2; ++nb) {
        f32x16 acc = {};
        for (int ks = 0; ks < MLP_NF / 8; ++ks) {
            bf16x4 a, b;
            for (int q = 0; q < 4; ++q) {
                a[q] = (short)B.x[lr * MLP_NF + ks * 8 + lk + q];
                b[q] = (short)W.w1[(nb * 32 + lr) * MLP_NF + ks * 8 + lk + q];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
        }
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r >> 2) + lk + (r & 3), j = nb * 32 + lr;
            const float z = acc[r] + W.b1[j];
            B.h1[i * MLP_NH + j] = f2bf(z > 0.f ? z : 0.f);
        }
    }
    __syncthreads();
    for (int nb = 0; nb < 2; ++nb) {
        f32x16 acc = {};
        for (int ks = 0; ks < MLP_NH / 8; ++ks) {
            bf16x4 a, b;
            for (int q = 0; q < 4; ++q) {
                a[q] = (short)B.h1[lr * MLP_NH + ks * 8 + lk + q];
                b[q] = (short)W.w2[(nb * 32 + lr) * MLP_NH + ks * 8 + lk + q];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
        }
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r >> 2) + lk + (r & 3), j = nb * 32 + lr;
            const float z = acc[r] + W.b2[j];
            B.h2[i * MLP_NH + j] = z > 0.f ? z : 0.f;
        }
    }
    __syncthreads();
}

}  // namespace

// ---------------------------------------------------------------------------
// edges and features
// ---------------------------------------------------------------------------

// per row: number of edges (P entries of F rows), and the coarse -> fine map
__global__ void k_edge_count(int n, const int *__restrict__ cf, const int *__restrict__ cidx,
                             const int *__restrict__ prp, int *__restrict__ cnt, int *__restrict__ isf,
                             int *__restrict__ fine_of) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int len = prp[i + 1] - prp[i];
    const bool f = (cf[i] == 0) && len > 0;
    cnt[i] = f ? len : 0;
    isf[i] = f ? 1 : 0;
    if (cf[i] == 1) fine_of[cidx[i]] = i;
}

__global__ void k_edge_rows(int n, const int *__restrict__ isf, const int *__restrict__ fpos,
                            const int *__restrict__ estart_row, int *__restrict__ frows, int *__restrict__ estart) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (isf[i]) {
        frows[fpos[i]] = i;
        estart[fpos[i]] = estart_row[i];
    }
    if (i == n - 1) estart[fpos[n]] = estart_row[n];   // closing entry (fpos[n] = number of F rows)
}

__device__ inline bool csr_entry(const int *rp, const int *ci, const double *v, int i, int j, double &out) {
    for (int e = rp[i]; e < rp[i + 1]; ++e)
        if (ci[e] == j) { out = v[e]; return true; }
    out = 0.0;
    return false;
}

__global__ void k_edge_features(int nf, const int *__restrict__ frows, const int *__restrict__ estart,
                                const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ v,
                                const unsigned char *__restrict__ strong, const int *__restrict__ prp,
                                const int *__restrict__ pci, const double *__restrict__ pv,
                                const int *__restrict__ fine_of, float *__restrict__ X) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nf) return;
    const int i = frows[q];
    const int lo = rp[i], hi = rp[i + 1];
    double aii = 0.0, rowsum = 0.0;
    int nstrong = 0;
    for (int e = lo; e < hi; ++e) {
        if (ci[e] == i) aii = v[e];
        rowsum += v[e];
        nstrong += strong[e] ? 1 : 0;
    }
    const double si = aii < 0.0 ? -1.0 : 1.0;
    double smax = 0.0;
    bool first = true;
    for (int e = lo; e < hi; ++e) {
        if (ci[e] == i) continue;
        const double t = -si * v[e];
        if (first || t > smax) smax = t;
        first = false;
    }
    if (first) smax = 0.0;
    const int plo = prp[i], phi = prp[i + 1];
    double S = 0.0, wmax = 0.0;
    bool wfirst = true;
    for (int e = plo; e < phi; ++e) {
        S += pv[e];
        const double a = fabs(pv[e]);
        if (wfirst || a > wmax) wmax = a;
        wfirst = false;
    }
    for (int e = plo; e < phi; ++e) {
        const int j = fine_of[pci[e]];
        double aij, aji, ajj;
        const bool present = csr_entry(rp, ci, v, i, j, aij);
        csr_entry(rp, ci, v, j, i, aji);
        csr_entry(rp, ci, v, j, j, ajj);
        double path = 0.0;
        for (int t = lo; t < hi; ++t) {
            const int k = ci[t];
            if (k == i || k == j) continue;
            double akj, akk;
            if (csr_entry(rp, ci, v, k, j, akj)) {
                csr_entry(rp, ci, v, k, k, akk);
                path += v[t] * akj / (aii * akk);
            }
        }
        double rowsum_j = 0.0;
        for (int t = rp[j]; t < rp[j + 1]; ++t) rowsum_j += v[t];
        const double den = fabs(aij) + fabs(aji);
        double x[MLP_NF];
        x[0] = aij / aii;
        x[1] = aji / ajj;
        x[2] = smax > 0.0 ? (-si * aij) / smax : 0.0;
        x[3] = present ? 0.0 : 1.0;
        x[4] = pv[e];
        x[5] = path;
        x[6] = rowsum / aii;
        x[7] = 1.0 / (double)(phi - plo);
        x[8] = den > 0.0 ? (aij - aji) / den : 0.0;
        x[9] = S;
        x[10] = wmax > 0.0 ? pv[e] / wmax : 0.0;
        x[11] = fabs(ajj) / (fabs(aii) + fabs(ajj));
        x[12] = rowsum_j / ajj;
        x[13] = (hi - lo > 1) ? (double)nstrong / (double)(hi - lo - 1) : 0.0;
        x[14] = 1.0;
        x[15] = 0.0;
        const long eo = (long)estart[q] + (e - plo);
        for (int f = 0; f < MLP_NF; ++f) X[eo * MLP_NF + f] = (float)x[f];
    }
}

// ---------------------------------------------------------------------------
// inference: o_e for every edge
// ---------------------------------------------------------------------------
// The layers are computed transposed, H_l^T = W_l H_{l-1}^T: hidden units are
// the MFMA rows, the tile's 32 edges the columns.  The accumulator of a
// 32 x 32 block then holds, in lane l, edge l % 32 and the rows
// 8 g + 4 (l / 32) + q (g, q = 0..3) -- exactly the B operand (k = 4 (l / 32)
// + q of K-step g) that the next layer's product over those rows takes, so
// the first hidden layer goes from one product to the next in registers.
// W1 and W2 stay in registers as A operands for the whole launch (row
// 32 m + l % 32, k = 8 s + 4 (l / 32) + q of K-step s); biases and W3 come
// from LDS (every half-wavefront reads one address).  One wavefront per tile
// at a time, tiles strided over the grid, the next tile's features loaded
// while the current one computes.
constexpr int FWD_WAVES = 4;
constexpr int FWD_MAX_BLOCKS = 512;

__global__ void __launch_bounds__(64 * FWD_WAVES) k_mlp_forward(int E, const float *__restrict__ X,
                                                                const float *__restrict__ params,
                                                                float *__restrict__ o) {
    __shared__ float b1s[MLP_NH], b2s[MLP_NH], w3s[MLP_NH];
    __shared__ float b3s;
    for (int k = threadIdx.x; k < MLP_NH; k += blockDim.x) {
        b1s[k] = params[OB1 + k];
        b2s[k] = params[OB2 + k];
        w3s[k] = bf2f(f2bf(params[OW3 + k]));
    }
    if (threadIdx.x == 0) b3s = params[OB3];
    const int lane = threadIdx.x & 63, lr = lane & 31, lk = 4 * (lane >> 5);
    bf16x4 a1[2][MLP_NF / 8], a2[2][MLP_NH / 8];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
#pragma unroll
        for (int ks = 0; ks < MLP_NF / 8; ++ks)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                a1[m][ks][q] = (short)f2bf(params[OW1 + (m * 32 + lr) * MLP_NF + ks * 8 + lk + q]);
#pragma unroll
        for (int ks = 0; ks < MLP_NH / 8; ++ks)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                a2[m][ks][q] = (short)f2bf(params[OW2 + (m * 32 + lr) * MLP_NH + ks * 8 + lk + q]);
    }
    __syncthreads();
    const long ntiles = ((long)E + TILE - 1) / TILE;
    const long stride = (long)gridDim.x * FWD_WAVES;
    long t = (long)blockIdx.x * FWD_WAVES + (threadIdx.x >> 6);
    // this lane's features of edge t * 32 + lr: [lk, lk + 4) and [8 + lk, 12 + lk)
    // (edges past the last one read as zeros)
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    long e = t * TILE + lr;
    float4 u = (e < E) ? reinterpret_cast<const float4 *>(X + e * MLP_NF)[lk / 4] : zero4;
    float4 v = (e < E) ? reinterpret_cast<const float4 *>(X + e * MLP_NF)[2 + lk / 4] : zero4;
    for (; t < ntiles; t += stride) {
        bf16x4 bx[2];
        bx[0][0] = (short)f2bf(u.x); bx[0][1] = (short)f2bf(u.y); bx[0][2] = (short)f2bf(u.z); bx[0][3] = (short)f2bf(u.w);
        bx[1][0] = (short)f2bf(v.x); bx[1][1] = (short)f2bf(v.y); bx[1][2] = (short)f2bf(v.z); bx[1][3] = (short)f2bf(v.w);
        const long en = (t + stride) * TILE + lr;       // the next tile's edge
        u = (en < E) ? reinterpret_cast<const float4 *>(X + en * MLP_NF)[lk / 4] : zero4;
        v = (en < E) ? reinterpret_cast<const float4 *>(X + en * MLP_NF)[2 + lk / 4] : zero4;
        // layer 1: H1^T (64 x 32) = W1 (64 x 16) X^T (16 x 32)
        f32x16 z1[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            z1[m] = f32x16{};
#pragma unroll
            for (int ks = 0; ks < MLP_NF / 8; ++ks)
                z1[m] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[m][ks], bx[ks], z1[m], 0, 0, 0);
        }
        // h1 = BF16(ReLU(z1 + b1)) as the B operands of layer 2's K-steps
        bf16x4 hb[MLP_NH / 8];
#pragma unroll
        for (int ks = 0; ks < MLP_NH / 8; ++ks)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = ks / 4, r = 4 * (ks % 4) + q;
                const float z = z1[m][r] + b1s[m * 32 + 8 * (ks % 4) + lk + q];
                hb[ks][q] = (short)f2bf(z > 0.f ? z : 0.f);
            }
        // layer 2: H2^T (64 x 32) = W2 (64 x 64) H1^T (64 x 32); output
        // o = W3 h2 + b3 (this lane's 32 rows, then the other half's)
        float part = 0.f;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            f32x16 z2 = {};
#pragma unroll
            for (int ks = 0; ks < MLP_NH / 8; ++ks)
                z2 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a2[m][ks], hb[ks], z2, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = m * 32 + 8 * (r >> 2) + lk + (r & 3);
                const float z = z2[r] + b2s[j];
                part += (z > 0.f ? z : 0.f) * w3s[j];
            }
        }
        const float tot = part + __shfl_xor(part, 32, 64);
        e = t * TILE + lr;
        if (lk == 0 && e < E) o[e] = tot + b3s;
    }
}

// ---------------------------------------------------------------------------
// learned weights and the training loss
// ---------------------------------------------------------------------------
constexpr int MAX_ROW_EDGES = 16;
constexpr int MAX_VECTORS = 16;

__device__ inline bool row_weights(int m, const double *w0, const double *delta, double *w, double &S, double &D) {
    S = 0.0;
    D = 0.0;
    for (int k = 0; k < m; ++k) {
        w[k] = w0[k] * (1.0 + delta[k]);
        S += w0[k];
        D += w[k];
    }
    if (D != 0.0) {
        const double c = S / D;
        if (c >= 0.25 && c <= 4.0) {
            for (int k = 0; k < m; ++k) w[k] = w[k] * S / D;
            return true;
        }
    }
    return false;
}

// per F row (one thread): the row's sums in a first pass over its edges, the
// weights in a second (the same expressions, in the same order, as the
// row_weights helper; pv_out may be pv)
__global__ void k_learned_weights(int nf, const int *__restrict__ frows, const int *__restrict__ estart,
                                  const int *__restrict__ prp, const double *pv, const float *__restrict__ o,
                                  double *pv_out) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nf) return;
    const int i = frows[q], plo = prp[i], e0 = estart[q];
    const int m = estart[q + 1] - e0;
    double S = 0.0, D = 0.0;
    for (int k = 0; k < m; ++k) {
        const double w0 = pv[plo + k];
        const double w = w0 * (1.0 + 0.5 * tanh((double)o[e0 + k]));
        S += w0;
        D += w;
    }
    bool scale = false;
    if (D != 0.0) {
        const double c = S / D;
        scale = (c >= 0.25 && c <= 4.0);
    }
    for (int k = 0; k < m; ++k) {
        const double w0 = pv[plo + k];
        double w = w0 * (1.0 + 0.5 * tanh((double)o[e0 + k]));
        if (scale) w = w * S / D;
        pv_out[plo + k] = w;
    }
}

// per F row: loss term and dL/do of its edges (E: K vectors of length n)
__global__ void k_interp_loss(int nf, int n, int K, const int *__restrict__ frows, const int *__restrict__ estart,
                              const int *__restrict__ prp, const int *__restrict__ pci, const double *__restrict__ pv,
                              const int *__restrict__ fine_of, const double *__restrict__ Ev,
                              const float *__restrict__ o, double *__restrict__ lossrow, float *__restrict__ dout) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nf) return;
    const int i = frows[q], plo = prp[i];
    const int m = estart[q + 1] - estart[q];
    double w0[MAX_ROW_EDGES], t[MAX_ROW_EDGES], d[MAX_ROW_EDGES], w[MAX_ROW_EDGES], g[MAX_ROW_EDGES], S, D;
    int jf[MAX_ROW_EDGES];
    for (int k = 0; k < m; ++k) {
        w0[k] = pv[plo + k];
        t[k] = tanh((double)o[estart[q] + k]);
        d[k] = 0.5 * t[k];
        jf[k] = fine_of[pci[plo + k]];
        g[k] = 0.0;
    }
    const bool scaled = row_weights(m, w0, d, w, S, D);
    double den = 0.0;
    for (int v = 0; v < K; ++v) den += Ev[(size_t)v * n + i] * Ev[(size_t)v * n + i];
    den += 1e-300;
    double loss = 0.0;
    for (int v = 0; v < K; ++v) {
        double r = Ev[(size_t)v * n + i];
        double s = 0.0;
        for (int k = 0; k < m; ++k) s += Ev[(size_t)v * n + jf[k]] * w[k];
        r = r - s;
        loss += r * r;
        for (int k = 0; k < m; ++k) g[k] += r * Ev[(size_t)v * n + jf[k]];
    }
    lossrow[q] = loss / den;
    double gw = 0.0;
    for (int k = 0; k < m; ++k) {
        g[k] = -2.0 * g[k] / den / (double)nf;
        gw += g[k] * w[k];
    }
    for (int k = 0; k < m; ++k) {
        const double dd = scaled ? (w0[k] / D) * (S * g[k] - gw) : g[k] * w0[k];
        dout[estart[q] + k] = (float)(dd * 0.5 * (1.0 - t[k] * t[k]));
    }
}

// smooth vectors: e <- e - omega (A e)_i / a_ii (zero right-hand side)
__global__ void k_jacobi_zero(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                              const double *__restrict__ v, double omega, const double *__restrict__ ein,
                              double *__restrict__ eout) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0, d = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
        acc += v[e] * ein[ci[e]];
        if (ci[e] == i) d = v[e];
    }
    eout[i] = ein[i] - omega * acc / d;
}

// ---------------------------------------------------------------------------
// backward pass: per-wavefront partial gradients of the parameter blob
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(THREADS) k_mlp_backward(int E, const float *__restrict__ X,
                                                          const float *__restrict__ params,
                                                          const float *__restrict__ dout,
                                                          float *__restrict__ part) {
    __shared__ Weights W;
    __shared__ WaveBuf Bw[WAVES];
    load_weights(params, W);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 31, lk = 4 * (lane >> 5);
    WaveBuf &B = Bw[wave];
    const long ntiles = ((long)E + TILE - 1) / TILE;
    const long groups = (ntiles + WAVES - 1) / WAVES;
    f32x16 gW2[2][2] = {}, gW1[2] = {};
    float gW3 = 0.f, gB2 = 0.f, gB1[2] = {0.f, 0.f}, gB3 = 0.f;
    __syncthreads();
    for (long gidx = blockIdx.x; gidx < groups; gidx += gridDim.x) {
        const long t = gidx * WAVES + wave;
        load_tile(lane, t, E, X, B);
        __syncthreads();
        forward_tile(lane, W, B);
        // output layer: lane j owns hidden unit j of the second layer
        {
            const int j = lane;
            for (int i = 0; i < TILE; ++i) {
                const long e = t * TILE + i;
                const float d = (e < E) ? dout[e] : 0.f;
                const float h2 = B.h2[i * MLP_NH + j];
                gW3 += d * h2;
                const float dz2 = (h2 > 0.f) ? d * W.w3[j] : 0.f;
                gB2 += dz2;
                B.d2[i * MLP_NH + j] = f2bf(dz2);
                if (j == 0) gB3 += d;
            }
        }
        __syncthreads();
        // dW2 += dz2^T h1 (M = h2 unit, N = h1 unit, K = edges)
        for (int mb = 0; mb < 2; ++mb)
            for (int nb = 0; nb < 2; ++nb)
                for (int ks = 0; ks < TILE / 8; ++ks) {
                    bf16x4 a, b;
                    for (int q = 0; q < 4; ++q) {
                        a[q] = (short)B.d2[(ks * 8 + lk + q) * MLP_NH + mb * 32 + lr];
                        b[q] = (short)B.h1[(ks * 8 + lk + q) * MLP_NH + nb * 32 + lr];
                    }
                    gW2[mb][nb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, gW2[mb][nb], 0, 0, 0);
                }
        // dh1 = dz2 W2, dz1 = dh1 [z1 > 0]
        for (int nb = 0; nb < 2; ++nb) {
            f32x16 acc = {};
            for (int ks = 0; ks < MLP_NH / 8; ++ks) {
                bf16x4 a, b;
                for (int q = 0; q < 4; ++q) {
                    a[q] = (short)B.d2[lr * MLP_NH + ks * 8 + lk + q];
                    b[q] = (short)W.w2[(ks * 8 + lk + q) * MLP_NH + nb * 32 + lr];
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
            }
            for (int r = 0; r < 16; ++r) {
                const int i = 8 * (r >> 2) + lk + (r & 3), j = nb * 32 + lr;
                const float dz1 = (B.h1[i * MLP_NH + j] != 0) ? acc[r] : 0.f;
                gB1[nb] += dz1;
                B.d1[i * MLP_NH + j] = f2bf(dz1);
            }
        }
        __syncthreads();
        // dW1 += dz1^T x (M = h1 unit, N = feature padded to 32, K = edges)
        for (int mb = 0; mb < 2; ++mb)
            for (int ks = 0; ks < TILE / 8; ++ks) {
                bf16x4 a, b;
                for (int q = 0; q < 4; ++q) {
                    a[q] = (short)B.d1[(ks * 8 + lk + q) * MLP_NH + mb * 32 + lr];
                    b[q] = (lr < MLP_NF) ? (short)B.x[(ks * 8 + lk + q) * MLP_NF + lr] : (short)0;
                }
                gW1[mb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, gW1[mb], 0, 0, 0);
            }
        __syncthreads();
    }
    // the wavefront's partial gradient, every parameter written once
    float *out = part + (size_t)(blockIdx.x * WAVES + wave) * MLP_NPARAMS;
    for (int mb = 0; mb < 2; ++mb)
        for (int r = 0; r < 16; ++r) {
            const int m = mb * 32 + 8 * (r >> 2) + lk + (r & 3);
            if (lr < MLP_NF) out[OW1 + m * MLP_NF + lr] = gW1[mb][r];
        }
    for (int mb = 0; mb < 2; ++mb)
        for (int nb = 0; nb < 2; ++nb)
            for (int r = 0; r < 16; ++r) {
                const int m = mb * 32 + 8 * (r >> 2) + lk + (r & 3), nn = nb * 32 + lr;
                out[OW2 + m * MLP_NH + nn] = gW2[mb][nb][r];
            }
    for (int nb = 0; nb < 2; ++nb) {
        const float s = gB1[nb] + __shfl_xor(gB1[nb], 32, 64);   // the two row halves of a column
        if (lane < 32) out[OB1 + nb * 32 + lr] = s;
    }
    out[OB2 + lane] = gB2;
    out[OW3 + lane] = gW3;
    if (lane == 0) out[OB3] = gB3;
}

// grad[p] = sum over wavefronts of part[w][p] (fixed order, FP64 sums)
__global__ void k_grad_reduce(int nw, const float *__restrict__ part, float *__restrict__ grad) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAMS) return;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += (double)part[(size_t)w * MLP_NPARAMS + p];
    grad[p] = (float)s;
}

// Adam (Kingma & Ba, Algorithm 1) on the FP32 master parameters
__global__ void k_adam(int np, float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, double lr, double b1, double b2, double eps, double c1,
                       double c2) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const double gk = g[k];
    const double mk = b1 * (double)m[k] + (1.0 - b1) * gk;
    const double vk = b2 * (double)v[k] + (1.0 - b2) * gk * gk;
    m[k] = (float)mk;
    v[k] = (float)vk;
    p[k] = (float)((double)p[k] - lr * (mk / c1) / (sqrt(vk / c2) + eps));
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
static inline int nblk(long n, int t) { long b = (n + t - 1) / t; return (int)(b < 1 ? 1 : b); }

void ln_edge_count(int n, const int *cf, const int *cidx, const int *prp, int *cnt, int *isf, int *fine_of,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_edge_count, dim3(nblk(n, 256)), dim3(256), 0, s, n, cf, cidx, prp, cnt, isf, fine_of);
    CPTR_CHECK_LAUNCH();
}

void ln_edge_rows(int n, const int *isf, const int *fpos, const int *estart_row, int *frows, int *estart,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_edge_rows, dim3(nblk(n, 256)), dim3(256), 0, s, n, isf, fpos, estart_row, frows, estart);
    CPTR_CHECK_LAUNCH();
}

void ln_edge_features(int nf, const int *frows, const int *estart, const int *rp, const int *ci, const double *v,
                      const unsigned char *strong, const int *prp, const int *pci, const double *pv,
                      const int *fine_of, float *X, hipStream_t s) {
    if (nf == 0) return;
    hipLaunchKernelGGL(k_edge_features, dim3(nblk(nf, 128)), dim3(128), 0, s, nf, frows, estart, rp, ci, v, strong,
                       prp, pci, pv, fine_of, X);
    CPTR_CHECK_LAUNCH();
}

static int mlp_grid(int E) {
    const long groups = ((long)E + TILE * WAVES - 1) / (TILE * WAVES);
    return (int)std::max(1L, std::min(groups, (long)MLP_MAX_BLOCKS));
}

int ln_mlp_waves(int E) { return mlp_grid(E) * WAVES; }

void ln_mlp_forward(int E, const float *X, const float *params, float *o, hipStream_t s) {
    if (E == 0) return;
    const long tiles = ((long)E + TILE - 1) / TILE;
    const int grid = (int)std::max(1L, std::min((tiles + FWD_WAVES - 1) / FWD_WAVES, (long)FWD_MAX_BLOCKS));
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(64 * FWD_WAVES), 0, s, E, X, params, o);
    CPTR_CHECK_LAUNCH();
}

void ln_learned_weights(int nf, const int *frows, const int *estart, const int *prp, const double *pv,
                        const float *o, double *pv_out, hipStream_t s) {
    if (nf == 0) return;
    hipLaunchKernelGGL(k_learned_weights, dim3(nblk(nf, 256)), dim3(256), 0, s, nf, frows, estart, prp, pv, o, pv_out);
    CPTR_CHECK_LAUNCH();
}

void ln_interp_loss(int nf, int n, int K, const int *frows, const int *estart, const int *prp, const int *pci,
                    const double *pv, const int *fine_of, const double *Ev, const float *o, double *lossrow,
                    float *dout, hipStream_t s) {
    if (nf == 0) return;
    hipLaunchKernelGGL(k_interp_loss, dim3(nblk(nf, 128)), dim3(128), 0, s, nf, n, K, frows, estart, prp, pci, pv,
                       fine_of, Ev, o, lossrow, dout);
    CPTR_CHECK_LAUNCH();
}

void ln_jacobi_zero(int n, const int *rp, const int *ci, const double *v, double omega, const double *ein,
                    double *eout, hipStream_t s) {
    hipLaunchKernelGGL(k_jacobi_zero, dim3(nblk(n, 256)), dim3(256), 0, s, n, rp, ci, v, omega, ein, eout);
    CPTR_CHECK_LAUNCH();
}

void ln_mlp_backward(int E, const float *X, const float *params, const float *dout, float *part, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_backward, dim3(mlp_grid(E)), dim3(THREADS), 0, s, E, X, params, dout, part);
    CPTR_CHECK_LAUNCH();
}

void ln_grad_reduce(int nw, const float *part, float *grad, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_reduce, dim3(nblk(MLP_NPARAMS, 256)), dim3(256), 0, s, nw, part, grad);
    CPTR_CHECK_LAUNCH();
}

void ln_adam(float *p, float *m, float *v, const float *g, double lr, double b1, double b2, double eps, int t,
             hipStream_t s) {
    const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
    hipLaunchKernelGGL(k_adam, dim3(nblk(MLP_NPARAMS, 256)), dim3(256), 0, s, MLP_NPARAMS, p, m, v, g, lr, b1, b2,
                       eps, c1, c2);
    CPTR_CHECK_LAUNCH();
}

}  // namespace cptr
