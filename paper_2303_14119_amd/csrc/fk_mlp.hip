// fk_mlp.hip -- the surrogate network: a multilayer perceptron with GELU
// hidden layers, trained on the GPU by hand-written BF16 MFMA GEMMs with FP32
// accumulation, fused bias / GELU / GELU' epilogues, an MSE loss kernel,
// bias-gradient reductions and an AdamW step on FP32 master weights.
//
// Every product is an "NT" GEMM, C[M][N] = A[M][K] * B[N][K]^T with both
// operands K-contiguous, so the operands of the three passes are stored in
// the layout they are read in:
//   forward   Z_l  = A_{l-1} W_l^T          A_{l-1} [M][K], W_l [N][K]
//   dgrad     dA_l = dZ_{l+1} (W_{l+1}^T)^T   dZ [M][N'], Wt_{l+1} [N][N'] (W transposed)
//   wgrad     dW_l = dZ_l^T (A_{l-1}^T)^T     dZt [N][M], At_{l-1} [K][M]
// The epilogues write activations and gradients in both layouts.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fk_internal.h"

namespace fk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kMaxLayers = 8;

enum GemmEpilogue {
    EPI_HIDDEN = 0,   // z = acc + b; store z (FP32), gelu(z) as bf16 [M][N] and [N][M]
    EPI_OUTPUT = 1,   // y = acc + b (FP32)
    EPI_DGRAD = 2,    // dz = acc * gelu'(z); store bf16 [M][N] and [N][M]
    EPI_WGRAD = 3,    // dW = acc (FP32)
    EPI_OUTPUT_LOSS = 4   // y = acc + b (FP32), dz = 2 (y - t) / (M dout) on the first dout columns, bf16 in
                          // both layouts, the tile's sum of squared errors to loss_part
};

struct GemmArgs {
    const __bf16* __restrict__ A;
    const __bf16* __restrict__ B;
    int lda, ldb;
    int M, N, K;                   // K a multiple of 16 (zero padded)
    const float* __restrict__ bias;
    const float* __restrict__ zin; // EPI_DGRAD: pre-activation of the layer
    int ldzin;
    float* __restrict__ out;       // FP32 output (z, y or dW)
    int ldout;
    __bf16* __restrict__ act;      // bf16 [M][N]
    int ldact;
    __bf16* __restrict__ actT;     // bf16 [N][M]
    int ldactT;
    int epi;
    const float* __restrict__ target;   // EPI_OUTPUT_LOSS: [M][dout]
    int dout;
    float gscale;                       // 2 / (M dout)
    double* __restrict__ loss_part;     // per-tile sums of squared errors
};

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// One launch runs one or two independent products (the weight and the input
// gradient of a layer need only its dZ): workgroups [0, tiles0) take tiles
// of p[0], the rest tiles of p[1]; ntn[i] is p[i]'s number of column tiles.
struct GemmPair {
    GemmArgs p[2];
    int tiles0;
    int ntn[2];
};

// One workgroup of 4 waves computes a 32 x 32 tile of C with
// v_mfma_f32_32x32x16_bf16, splitting K: wave w takes the K steps
// w, w + 4, w + 8, ... (16 each), so each wave's chain of dependent loads is
// a quarter of K; the four partial tiles are summed through LDS (fixed
// order), each wave finishing a quarter of the tile's elements.  Lane l
// holds A[row l%32][k0 + 8(l/32) .. +7] and B[col l%32][same k] and
// accumulates C element e at row 8(e/4) + 4(l/32) + e%4, column l%32 of the
// tile.  On return v[i] (i < 4) is the element at row m0 + 8w + 4(l/32) + i,
// column n0 + l%32.  Every thread of the workgroup calls it (one barrier).
constexpr int kGemmTile = 32;

// The first layer's A operand can come straight from the FP32 features
// x [M][dx] (zero past column dx, rounded to bf16 as k_mlp_input does)
// instead of a bf16 copy, which saves the training step the input launch;
// the tiles of the first column block then store that copy in both layouts
// (a [M][lda], at [lda][ldat]) for the first layer's weight gradient.
struct XIn {
    const float* x;
    int dx;
    __bf16* a;
    int lda;
    __bf16* at;
    int ldat;
};

template <bool XIN = false>
__device__ __forceinline__ void gemm_nt_tile(const GemmArgs& g, int m0, int n0, float (&part)[4][16][64],
                                             float (&v)[4], const XIn& xi = XIn{})
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int ra = m0 + (lane & 31), rb = n0 + (lane & 31);
    const int kk = 8 * (lane >> 5);
    const bool a_ok = ra < g.M, b_ok = rb < g.N;
    const __bf16* pa = g.A + (size_t)(a_ok ? ra : 0) * g.lda + kk;
    const __bf16* pb = g.B + (size_t)(b_ok ? rb : 0) * g.ldb + kk;
    f32x16 acc = {0};
    const bf16x8 zero = {0};
    // The wave's K steps (every fourth of 16) in groups of 8: all 16 operand
    // loads of a group are issued before its first MFMA, so a group costs one
    // memory latency.  Loads are unconditional (rows outside the matrix read
    // row 0, steps past the end repeat the last one) and the values are
    // zeroed or skipped afterwards; the MFMAs run in K order.
    const int nsteps = g.K > 16 * w ? (g.K - 16 * w + 63) / 64 : 0;
    for (int s0 = 0; s0 < nsteps; s0 += 8) {
        bf16x8 av[8], bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k0 = 16 * w + 64 * min(s0 + u, nsteps - 1);
            if constexpr (XIN) {
                const float* px = xi.x + (size_t)(a_ok ? ra : 0) * xi.dx;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int k = k0 + kk + i;
                    const float f = px[min(k, xi.dx - 1)];
                    av[u][i] = (__bf16)(k < xi.dx ? f : 0.0f);
                }
            } else {
                av[u] = *reinterpret_cast<const bf16x8*>(pa + k0);
            }
            bv[u] = *reinterpret_cast<const bf16x8*>(pb + k0);
        }
        if constexpr (XIN) {
            if (n0 == 0 && a_ok) {
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (s0 + u < nsteps) {
                        const int k = 16 * w + 64 * (s0 + u) + kk;
                        *reinterpret_cast<bf16x8*>(xi.a + (size_t)ra * xi.lda + k) = av[u];
#pragma unroll
                        for (int i = 0; i < 8; ++i) xi.at[(size_t)(k + i) * xi.ldat + ra] = av[u][i];
                    }
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (s0 + u < nsteps)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_ok ? av[u] : zero, b_ok ? bv[u] : zero, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 16; ++e) part[w][e][lane] = acc[e];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        // the four waves' partial sums, added in wave order
        const int e = 4 * w + i;
        v[i] = ((part[0][e][lane] + part[1][e][lane]) + part[2][e][lane]) + part[3][e][lane];
    }
}

template <bool XIN = false>
__global__ void __launch_bounds__(256) k_gemm_nt(GemmPair gp, XIn xi)
{
    __shared__ float part[4][16][64];       // every wave's partial tile: [wave][element][lane]
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int second = (int)blockIdx.x >= gp.tiles0 ? 1 : 0;
    const GemmArgs& g = gp.p[second];
    const int t = (int)blockIdx.x - (second ? gp.tiles0 : 0);
    const int m0 = (t / gp.ntn[second]) * kGemmTile;
    const int n0 = (t % gp.ntn[second]) * kGemmTile;
    // This thread finishes rows m0 + 8w + 4 (lane / 32) + i, column
    // n0 + lane % 32: their bias and pre-activation operands are loaded now,
    // alongside the first operand group, not after the reduction.
    const int col = n0 + (lane & 31);
    const bool col_ok = col < g.N;
    float bias_c = 0.0f, zpre[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (col_ok) {
        if (g.epi == EPI_HIDDEN || g.epi == EPI_OUTPUT || g.epi == EPI_OUTPUT_LOSS) bias_c = g.bias[col];
        if (g.epi == EPI_DGRAD) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = m0 + 8 * w + 4 * (lane >> 5) + i;
                zpre[i] = g.zin[(size_t)min(row, g.M - 1) * g.ldzin + col];
            }
        }
    }
    float vv[4];
    gemm_nt_tile<XIN>(g, m0, n0, part, vv, xi);
    if (g.epi == EPI_OUTPUT_LOSS) {
        // every thread reaches the workgroup sum below
        __shared__ double sq_w[4];
        double sq = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = m0 + 8 * w + 4 * (lane >> 5) + i;
            if (!col_ok || row >= g.M) continue;
            const float y = vv[i] + bias_c;
            g.out[(size_t)row * g.ldout + col] = y;
            float gr = 0.0f;
            if (col < g.dout) {
                const float d = y - g.target[(size_t)row * g.dout + col];
                sq += (double)d * d;
                gr = g.gscale * d;
            }
            const __bf16 h = (__bf16)gr;
            g.act[(size_t)row * g.ldact + col] = h;
            g.actT[(size_t)col * g.ldactT + row] = h;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, 64);
        if (lane == 0) sq_w[w] = sq;
        __syncthreads();
        if (threadIdx.x == 0) g.loss_part[t] = ((sq_w[0] + sq_w[1]) + sq_w[2]) + sq_w[3];
        return;
    }
    if (!col_ok) return;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = m0 + 8 * w + 4 * (lane >> 5) + i;
        if (row >= g.M) continue;
        const float v = vv[i];
        switch (g.epi) {
        case EPI_HIDDEN: {
            const float z = v + bias_c;
            g.out[(size_t)row * g.ldout + col] = z;
            const __bf16 h = (__bf16)gelu(z);
            g.act[(size_t)row * g.ldact + col] = h;
            g.actT[(size_t)col * g.ldactT + row] = h;
            break;
        }
        case EPI_OUTPUT:
            g.out[(size_t)row * g.ldout + col] = v + bias_c;
            break;
        case EPI_DGRAD: {
            const __bf16 d = (__bf16)(v * gelu_grad(zpre[i]));
            g.act[(size_t)row * g.ldact + col] = d;
            g.actT[(size_t)col * g.ldactT + row] = d;
            break;
        }
        default:
            g.out[(size_t)row * g.ldout + col] = v;
            break;
        }
    }
}

// Fixed-order workgroup sum (blockDim.x a power of two, <= 1024).
__device__ double mlp_block_sum(double v, double* sh)
{
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    return sh[0];
}

// Input: FP32 [M][d] -> bf16 [M][ld] and [ld][M]-transposed, zero padded.
__global__ void k_mlp_input(const float* __restrict__ x, int M, int d, int pad, __bf16* __restrict__ a, int lda,
                            __bf16* __restrict__ at, int ldat)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * pad) return;
    const int m = idx / pad, k = idx % pad;
    const __bf16 v = (__bf16)(k < d ? x[(size_t)m * d + k] : 0.0f);
    a[(size_t)m * lda + k] = v;
    at[(size_t)k * ldat + m] = v;
}

// MSE loss over the first dout columns and its gradient 2 (y - t) / (M dout)
// as bf16 in both layouts (padded columns get 0).  Workgroup b takes rows
// [kLossRows b, kLossRows (b + 1)) and writes its sum of squares to part[b].
constexpr int kLossRows = 4;

__global__ void __launch_bounds__(256) k_mlp_loss(const float* __restrict__ y, int ldy, const float* __restrict__ t,
                                                  int M, int dout, int pad, __bf16* __restrict__ dz, int lddz,
                                                  __bf16* __restrict__ dzt, int lddzt, double* __restrict__ part)
{
    __shared__ double sh[256];
    const double scale = 1.0 / ((double)M * dout);
    const int m0 = blockIdx.x * kLossRows;
    const int rows = min(kLossRows, M - m0);
    double acc = 0.0;
    for (int idx = threadIdx.x; idx < rows * pad; idx += blockDim.x) {
        const int m = m0 + idx / pad, n = idx % pad;
        float g = 0.0f;
        if (n < dout) {
            const float r = y[(size_t)m * ldy + n] - t[(size_t)m * dout + n];
            acc += (double)r * r;
            g = (float)(2.0 * scale) * r;
        }
        const __bf16 h = (__bf16)g;
        dz[(size_t)m * lddz + n] = h;
        dzt[(size_t)n * lddzt + m] = h;
    }
    acc = mlp_block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// loss = scale * sum of the partials, in a fixed order (one workgroup); the
// loss is also added to the running sum acc[0] and acc[1] counts the steps
__global__ void __launch_bounds__(256) k_mlp_loss_sum(const double* __restrict__ part, int n, double scale,
                                                      float* __restrict__ loss, double* __restrict__ acc_sum)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
    acc = mlp_block_sum(acc, sh);
    if (threadIdx.x == 0) {
        const float l = (float)(acc * scale);
        *loss = l;
        acc_sum[0] += (double)l;
        acc_sum[1] += 1.0;
    }
}

// Bias gradients of every layer in one launch: db_l[n] = sum_m dz_l[m][n]
// from the transposed copies, one wave per n (fixed order: strided lane
// sums, then the wave's butterfly).  Layer s has workgroups
// [first[s], first[s + 1]), four columns each.
struct BiasArgs {
    const __bf16* dzt[kMaxLayers];
    float* db[kMaxLayers];
    int n[kMaxLayers];
    int first[kMaxLayers + 1];
    int nseg, lddzt, M;
};

__global__ void __launch_bounds__(256) k_mlp_bias_grad(BiasArgs a)
{
    int s = 0;
    while (s + 1 < a.nseg && (int)blockIdx.x >= a.first[s + 1]) ++s;
    const int n = ((int)blockIdx.x - a.first[s]) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (n >= a.n[s]) return;
    const __bf16* dzt = a.dzt[s];
    float acc = 0.0f;
    for (int m = lane; m < a.M; m += 64) acc += (float)dzt[(size_t)n * a.lddzt + m];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) a.db[s][n] = acc;
}

// AdamW (decoupled weight decay) on FP32 master weights, every tensor of the
// network in one launch.  Segment s is a weight matrix [N][ld] (refreshing
// its bf16 copies [N][ld] and [ld][ldT]) or a bias (wbf == nullptr, no
// decay); its workgroups are blocks [first[s], first[s + 1]).
constexpr int kAdamMaxSegs = 2 * kMaxLayers;

struct AdamSeg {
    float* w;
    const float* g;
    float* m;
    float* v;
    __bf16* wbf;
    __bf16* wtbf;
    int ld, ldT, count;
    float wd;
};

struct AdamArgs {
    AdamSeg seg[kAdamMaxSegs];
    int first[kAdamMaxSegs + 1];
    int nseg;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1 - b1^t, c2 = 1 - b2^t
};

// One AdamW update of element idx from its gradient g; returns the new weight.
__device__ __forceinline__ float adam_step(float lr, float b1, float b2, float eps, float c1, float c2, float wd,
                                           float g, float* wp, float* mp, float* vp, int idx)
{
    const float m = b1 * mp[idx] + (1.0f - b1) * g;
    const float v = b2 * vp[idx] + (1.0f - b2) * g * g;
    mp[idx] = m;
    vp[idx] = v;
    const float mh = m / c1, vh = v / c2;
    float w = wp[idx];
    w -= lr * (mh / (sqrtf(vh) + eps) + wd * w);
    wp[idx] = w;
    return w;
}

__device__ __forceinline__ float adamw_update(const AdamArgs& a, const AdamSeg& q, int idx)
{
    return adam_step(a.lr, a.b1, a.b2, a.eps, a.c1, a.c2, q.wd, q.g[idx], q.w, q.m, q.v, idx);
}

// A weight segment is covered by 32 x 32 tiles, one per workgroup: the
// update and the row-major bf16 copy go out along rows, and the transposed
// copy is staged through LDS so that it too is written in runs of
// consecutive addresses.  A bias segment is a plain range of 256 per
// workgroup.
__global__ void __launch_bounds__(256) k_adamw(AdamArgs a)
{
    __shared__ __attribute__((aligned(16))) __bf16 tile_t[32][36];   // [column][row]; rows 8-byte aligned
    int s = 0;
    while (s + 1 < a.nseg && (int)blockIdx.x >= a.first[s + 1]) ++s;
    const AdamSeg& q = a.seg[s];
    const int blk = (int)blockIdx.x - a.first[s];
    if (!q.wbf) {
        const int idx = blk * blockDim.x + threadIdx.x;
        if (idx < q.count) adamw_update(a, q, idx);
        return;
    }
    const int rows = q.count / q.ld;
    const int ntc = (q.ld + 31) / 32;
    const int r0 = (blk / ntc) * 32, c0 = (blk % ntc) * 32;
    const int cc = threadIdx.x & 31, rg = threadIdx.x >> 5;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int rr = rg + 8 * i, r = r0 + rr, c = c0 + cc;
        __bf16 h = (__bf16)0.0f;
        if (r < rows && c < q.ld) {
            const int idx = r * q.ld + c;
            h = (__bf16)adamw_update(a, q, idx);
            q.wbf[idx] = h;
        }
        tile_t[cc][rr] = h;
    }
    __syncthreads();
    // transposed copy: thread -> column c0 + t / 8, rows r0 + 4 (t % 8) .. + 3
    const int c = c0 + (threadIdx.x >> 3), rq = 4 * (threadIdx.x & 7);
    if (c < q.ld && r0 + rq < rows) {
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 v = *reinterpret_cast<const u32x2*>(&tile_t[threadIdx.x >> 3][rq]);
        *reinterpret_cast<u32x2*>(q.wtbf + (size_t)c * q.ldT + r0 + rq) = v;
    }
}

// Refresh the bf16 copies of a weight matrix from its FP32 master.
__global__ void k_weight_copies(const float* __restrict__ w, int count, int ld, int ldT, __bf16* __restrict__ wbf,
                                __bf16* __restrict__ wtbf)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    const int r = idx / ld, c = idx % ld;
    wbf[idx] = (__bf16)w[idx];
    wtbf[(size_t)c * ldT + r] = (__bf16)w[idx];
}


// ---------------------------------------------------------- training step
// A whole training step in fewer launches (fk_mlp_train_step): the forward
// GEMMs (the first reading the FP32 features itself), the output GEMM with
// the loss and its gradient in its epilogue
// (per-tile sums of squared errors), the input-gradient GEMMs, then one
// launch for every weight gradient dW_l = dZ_{l+1}^T A_l as 32 x 32 tiles
// (K = the batch, the four-wave tile of k_gemm_nt), each tile written and
// updated by AdamW in its epilogue (FP32 master, moments, both bf16
// copies), one workgroup per four bias entries (the gradient from dZ^T,
// AdamW) and one for the loss.

// Four bf16 values of consecutive rows r0 .. r0 + 3 of a column, stored to a
// transposed [n][m] array at dst (8-byte aligned) when all four rows exist.
__device__ __forceinline__ void store_col4(__bf16* dst, const __bf16 (&h)[4], int nrows)
{
    if (nrows >= 4) {
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 v = {h[0], h[1], h[2], h[3]};
        *reinterpret_cast<bf16x4*>(dst) = v;
    } else {
        for (int i = 0; i < nrows; ++i) dst[i] = h[i];
    }
}

struct WgradAdamArgs {
    GemmArgs p[kMaxLayers];             // dW_l: A = dZ_{l+1}^T [pad[l+1]][mb], B = A_l^T [pad[l]][mb], K = M
    int ntn[kMaxLayers];
    int first[kMaxLayers + 1];          // workgroup ranges of the weight tiles
    AdamSeg wseg[kMaxLayers];           // the weights' state (g unused)
    AdamSeg bseg[kMaxLayers];           // the biases' state (g unused)
    float* wgrad[kMaxLayers];           // out: the weight gradients [pad[l+1]][pad[l]]
    float* bgrad[kMaxLayers];           // out: the bias gradients
    int bfirst[kMaxLayers + 1];         // workgroup ranges of the biases (after the tiles), 4 entries each
    int nl, nloss;
    const double* loss_part;            // [nloss]
    double loss_scale;                  // 1 / (M dout)
    float* loss;
    double* loss_acc;
    float lr, b1, b2, eps, c1, c2;
};

__global__ void __launch_bounds__(256) k_mlp_wgrad_adam(WgradAdamArgs a)
{
    __shared__ float part[4][16][64];
    const int bid = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (bid < a.first[a.nl]) {
        int s = 0;
        while (s + 1 < a.nl && bid >= a.first[s + 1]) ++s;
        const GemmArgs& g = a.p[s];
        const int tt = bid - a.first[s];
        const int m0 = (tt / a.ntn[s]) * kGemmTile, n0 = (tt % a.ntn[s]) * kGemmTile;
        float v[4];
        gemm_nt_tile(g, m0, n0, part, v);
        const AdamSeg& q = a.wseg[s];
        const int col = n0 + (lane & 31);
        if (col >= g.N) return;
        const int r0 = m0 + 8 * w + 4 * (lane >> 5);
        __bf16 h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            h[i] = (__bf16)0.0f;
            const int row = r0 + i;
            if (row >= g.M) continue;
            const int idx = row * q.ld + col;
            a.wgrad[s][idx] = v[i];
            const float wn = adam_step(a.lr, a.b1, a.b2, a.eps, a.c1, a.c2, q.wd, v[i], q.w, q.m, q.v, idx);
            h[i] = (__bf16)wn;
            q.wbf[idx] = h[i];
        }
        store_col4(q.wtbf + (size_t)col * q.ldT + r0, h, g.M - r0);
        return;
    }
    const int bb = bid - a.first[a.nl];
    if (bb < a.bfirst[a.nl]) {
        // four bias entries per workgroup, one wave each: the gradient
        // db_l[n] = sum_m dZ_{l+1}[m][n] from the transposed copy (strided
        // lane sums, then the wave's butterfly, as k_mlp_bias_grad), then
        // AdamW without decay
        int s = 0;
        while (s + 1 < a.nl && bb >= a.bfirst[s + 1]) ++s;
        const AdamSeg& q = a.bseg[s];
        const int n = (bb - a.bfirst[s]) * 4 + w;
        if (n >= q.count) return;
        const __bf16* dzt = a.p[s].A + (size_t)n * a.p[s].lda;
        float acc = 0.0f;
        for (int m = lane; m < a.p[s].K; m += 64) acc += (float)dzt[m];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) {
            a.bgrad[s][n] = acc;
            adam_step(a.lr, a.b1, a.b2, a.eps, a.c1, a.c2, 0.0f, acc, q.w, q.m, q.v, n);
        }
        return;
    }
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int b = 0; b < a.nloss; ++b) acc += a.loss_part[b];
        const float l = (float)(acc * a.loss_scale);
        *a.loss = l;
        a.loss_acc[0] += (double)l;
        a.loss_acc[1] += 1.0;
    }
}

}  // namespace fk

using namespace fk;

struct fk_mlp {
    int L = 0;
    int dims[kMaxLayers + 1] = {0};
    int pad[kMaxLayers + 1] = {0};      // dims[0] padded to 16, others to 32
    int max_batch = 0;
    int last_m = -1;                     // batch of the last forward
    hipStream_t stream = nullptr;
    void* pool = nullptr;
    float *w[kMaxLayers], *b[kMaxLayers], *gw[kMaxLayers], *gb[kMaxLayers];
    float *mw[kMaxLayers], *vw[kMaxLayers], *mb[kMaxLayers], *vb[kMaxLayers];
    __bf16 *wbf[kMaxLayers], *wtbf[kMaxLayers];
    __bf16 *act[kMaxLayers + 1], *actT[kMaxLayers + 1];
    float* z[kMaxLayers + 1];
    __bf16 *dz[kMaxLayers + 1], *dzT[kMaxLayers + 1];
    float* loss = nullptr;
    double* loss_part = nullptr;         // per-workgroup sums of squares
    double* loss_acc = nullptr;          // [2]: sum of the step losses since the last take, steps
    std::string err;
};

namespace {

int mfail(fk_mlp* n, hipError_t e, const char* what)
{
    return set_error(n ? &n->err : nullptr, FK_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define FK_MHIP(n, call)                                    \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return mfail((n), e_, #call); \
    } while (0)

int round_up(int v, int m) { return (v + m - 1) / m * m; }

int gemm_tiles(const GemmArgs& g, int* ntn)
{
    *ntn = (g.N + kGemmTile - 1) / kGemmTile;
    return *ntn * ((g.M + kGemmTile - 1) / kGemmTile);
}

// one product, or two independent ones in the same launch; with xi the
// first layer's product reading the FP32 features itself
void launch_gemm(const fk_mlp* n, const GemmArgs& g, const GemmArgs* g2 = nullptr, const XIn* xi = nullptr)
{
    GemmPair gp{};
    gp.p[0] = g;
    gp.tiles0 = gemm_tiles(g, &gp.ntn[0]);
    int tiles = gp.tiles0;
    if (g2) {
        gp.p[1] = *g2;
        tiles += gemm_tiles(*g2, &gp.ntn[1]);
    } else {
        gp.ntn[1] = 1;
    }
    if (xi) hipLaunchKernelGGL(k_gemm_nt<true>, dim3(tiles), dim3(256), 0, n->stream, gp, *xi);
    else hipLaunchKernelGGL(k_gemm_nt<false>, dim3(tiles), dim3(256), 0, n->stream, gp, XIn{});
}

}  // namespace

extern "C" int fk_mlp_create(int n_layers, const int32_t* dims, int max_batch, void* stream, fk_mlp** out)
{
    if (!out || !dims || n_layers < 1 || n_layers > kMaxLayers || max_batch < 16 || max_batch % 16)
        return set_error(nullptr, FK_E_INVALID, "fk_mlp_create: 1..8 layers and max_batch a positive multiple of 16");
    for (int l = 0; l <= n_layers; ++l)
        if (dims[l] < 1 || dims[l] > 8192) return set_error(nullptr, FK_E_INVALID, "fk_mlp_create: widths in [1, 8192]");
    fk_mlp* n = new (std::nothrow) fk_mlp();
    if (!n) return set_error(nullptr, FK_E_OOM, "host allocation failed");
    n->L = n_layers;
    n->max_batch = max_batch;
    n->stream = static_cast<hipStream_t>(stream);
    for (int l = 0; l <= n_layers; ++l) {
        n->dims[l] = dims[l];
        n->pad[l] = l == 0 ? round_up(dims[l], 16) : round_up(dims[l], 32);
    }
    // one pool: parameters, gradients, moments, bf16 copies, activations
    size_t off = 0;
    std::vector<std::pair<void**, size_t>> want;
    auto need = [&](void** p, size_t bytes) { want.push_back({p, bytes}); };
    const size_t M = max_batch;
    for (int l = 0; l < n_layers; ++l) {
        const size_t wn = (size_t)n->pad[l + 1] * n->pad[l], bn = n->pad[l + 1];
        need((void**)&n->w[l], wn * 4); need((void**)&n->gw[l], wn * 4);
        need((void**)&n->mw[l], wn * 4); need((void**)&n->vw[l], wn * 4);
        need((void**)&n->b[l], bn * 4); need((void**)&n->gb[l], bn * 4);
        need((void**)&n->mb[l], bn * 4); need((void**)&n->vb[l], bn * 4);
        need((void**)&n->wbf[l], wn * 2); need((void**)&n->wtbf[l], wn * 2);
    }
    for (int l = 0; l <= n_layers; ++l) {
        need((void**)&n->act[l], M * n->pad[l] * 2); need((void**)&n->actT[l], M * n->pad[l] * 2);
        need((void**)&n->z[l], M * n->pad[l] * 4);
        need((void**)&n->dz[l], M * n->pad[l] * 2); need((void**)&n->dzT[l], M * n->pad[l] * 2);
    }
    need((void**)&n->loss, 256);
    need((void**)&n->loss_acc, 256);
    // per-workgroup sums of squared errors: the loss kernel's row groups or
    // the output tiles of the training step's output GEMM
    const size_t out_tiles = ((M + kGemmTile - 1) / kGemmTile) * ((n->pad[n_layers] + kGemmTile - 1) / kGemmTile);
    need((void**)&n->loss_part, std::max<size_t>((M + kLossRows - 1) / kLossRows, out_tiles) * sizeof(double));
    for (auto& q : want) off += (q.second + 255) & ~size_t(255);
    if (hipMalloc(&n->pool, off) != hipSuccess) {
        delete n;
        return set_error(nullptr, FK_E_OOM, "device allocation of the network failed");
    }
    char* base = static_cast<char*>(n->pool);
    off = 0;
    for (auto& q : want) {
        *q.first = base + off;
        off += (q.second + 255) & ~size_t(255);
    }
    if (hipMemsetAsync(n->pool, 0, off, n->stream) != hipSuccess || hipStreamSynchronize(n->stream) != hipSuccess) {
        (void)hipFree(n->pool);
        delete n;
        return set_error(nullptr, FK_E_HIP, "clearing the network memory failed");
    }
    *out = n;
    return FK_OK;
}

extern "C" int fk_mlp_destroy(fk_mlp* n)
{
    if (!n) return FK_E_INVALID;
    (void)hipStreamSynchronize(n->stream);
    if (n->pool) (void)hipFree(n->pool);
    delete n;
    return FK_OK;
}

extern "C" const char* fk_mlp_last_error(const fk_mlp* n) { return n ? n->err.c_str() : global_error(); }

extern "C" int fk_mlp_num_params(const fk_mlp* n, int64_t* count)
{
    if (!n || !count) return FK_E_INVALID;
    int64_t c = 0;
    for (int l = 0; l < n->L; ++l) c += (int64_t)n->dims[l + 1] * n->dims[l] + n->dims[l + 1];
    *count = c;
    return FK_OK;
}

namespace {

// copy between the flat [W_1 (out x in), b_1, W_2, b_2, ...] vector and the
// padded device arrays; which = 0: parameters, 1: gradients
int flat_copy(fk_mlp* n, float* flat, int on_device, int which, bool to_net)
{
    const hipMemcpyKind kind = to_net ? (on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice)
                                      : (on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
    size_t off = 0;
    for (int l = 0; l < n->L; ++l) {
        const int in = n->dims[l], outd = n->dims[l + 1], ld = n->pad[l];
        float* wd = which ? n->gw[l] : n->w[l];
        float* bd = which ? n->gb[l] : n->b[l];
        if (to_net)
            FK_MHIP(n, hipMemcpy2DAsync(wd, ld * 4, flat + off, in * 4, in * 4, outd, kind, n->stream));
        else
            FK_MHIP(n, hipMemcpy2DAsync(flat + off, in * 4, wd, ld * 4, in * 4, outd, kind, n->stream));
        off += (size_t)in * outd;
        if (to_net) FK_MHIP(n, hipMemcpyAsync(bd, flat + off, outd * 4, kind, n->stream));
        else FK_MHIP(n, hipMemcpyAsync(flat + off, bd, outd * 4, kind, n->stream));
        off += outd;
        if (to_net && which == 0) {
            const int count = n->pad[l + 1] * ld;
            hipLaunchKernelGGL(k_weight_copies, dim3((count + 255) / 256), dim3(256), 0, n->stream, n->w[l], count,
                               ld, n->pad[l + 1], n->wbf[l], n->wtbf[l]);
        }
    }
    FK_MHIP(n, hipStreamSynchronize(n->stream));
    return FK_OK;
}

}  // namespace

extern "C" int fk_mlp_set_params(fk_mlp* n, const float* src, int src_on_device)
{
    if (!n || !src) return FK_E_INVALID;
    return flat_copy(n, const_cast<float*>(src), src_on_device, 0, true);
}

extern "C" int fk_mlp_get_params(fk_mlp* n, float* dst, int dst_on_device)
{
    if (!n || !dst) return FK_E_INVALID;
    return flat_copy(n, dst, dst_on_device, 0, false);
}

extern "C" int fk_mlp_get_grads(fk_mlp* n, float* dst, int dst_on_device)
{
    if (!n || !dst) return FK_E_INVALID;
    return flat_copy(n, dst, dst_on_device, 1, false);
}

extern "C" int fk_mlp_forward(fk_mlp* n, const float* x, int M, float* y)
{
    if (!n || !x || M < 1 || M > n->max_batch) return set_error(n ? &n->err : nullptr, FK_E_INVALID, "bad fk_mlp_forward arguments");
    const int mb = n->max_batch;
    {
        const int count = M * n->pad[0];
        hipLaunchKernelGGL(k_mlp_input, dim3((count + 255) / 256), dim3(256), 0, n->stream, x, M, n->dims[0],
                           n->pad[0], n->act[0], n->pad[0], n->actT[0], mb);
    }
    for (int l = 0; l < n->L; ++l) {
        GemmArgs g{};
        g.A = n->act[l];
        g.lda = n->pad[l];
        g.B = n->wbf[l];
        g.ldb = n->pad[l];
        g.M = M;
        g.N = n->pad[l + 1];
        g.K = n->pad[l];
        g.bias = n->b[l];
        g.out = n->z[l + 1];
        g.ldout = n->pad[l + 1];
        g.act = n->act[l + 1];
        g.ldact = n->pad[l + 1];
        g.actT = n->actT[l + 1];
        g.ldactT = mb;
        g.epi = l + 1 < n->L ? EPI_HIDDEN : EPI_OUTPUT;
        launch_gemm(n, g);
    }
    if (y)
        FK_MHIP(n, hipMemcpy2DAsync(y, n->dims[n->L] * 4, n->z[n->L], n->pad[n->L] * 4, n->dims[n->L] * 4, M,
                                    hipMemcpyDeviceToDevice, n->stream));
    FK_MHIP(n, hipGetLastError());
    n->last_m = M;
    return FK_OK;
}

extern "C" int fk_mlp_backward(fk_mlp* n, const float* target, int M, float* loss_host)
{
    if (!n || !target || M != n->last_m || M % 16)
        return set_error(n ? &n->err : nullptr, FK_E_INVALID, "fk_mlp_backward needs the batch of the last forward (a multiple of 16)");
    const int mb = n->max_batch, L = n->L;
    const int loss_blocks = (M + kLossRows - 1) / kLossRows;
    hipLaunchKernelGGL(k_mlp_loss, dim3(loss_blocks), dim3(256), 0, n->stream, n->z[L], n->pad[L], target, M,
                       n->dims[L], n->pad[L], n->dz[L], n->pad[L], n->dzT[L], mb, n->loss_part);
    hipLaunchKernelGGL(k_mlp_loss_sum, dim3(1), dim3(256), 0, n->stream, n->loss_part, loss_blocks,
                       1.0 / ((double)M * n->dims[L]), n->loss, n->loss_acc);
    for (int l = L; l >= 1; --l) {
        // weight and bias gradients of layer l (1-based): dW = dZ_l^T A_{l-1}
        GemmArgs g{};
        g.A = n->dzT[l];
        g.lda = mb;
        g.B = n->actT[l - 1];
        g.ldb = mb;
        g.M = n->pad[l];
        g.N = n->pad[l - 1];
        g.K = M;
        g.out = n->gw[l - 1];
        g.ldout = n->pad[l - 1];
        g.epi = EPI_WGRAD;
        if (l == 1) launch_gemm(n, g);
        if (l > 1) {
            // gradient of the pre-activation of layer l-1: dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})
            GemmArgs d{};
            d.A = n->dz[l];
            d.lda = n->pad[l];
            d.B = n->wtbf[l - 1];
            d.ldb = n->pad[l];
            d.M = M;
            d.N = n->pad[l - 1];
            d.K = n->pad[l];
            d.zin = n->z[l - 1];
            d.ldzin = n->pad[l - 1];
            d.act = n->dz[l - 1];
            d.ldact = n->pad[l - 1];
            d.actT = n->dzT[l - 1];
            d.ldactT = mb;
            d.epi = EPI_DGRAD;
            launch_gemm(n, g, &d);
        }
    }
    {
        // the bias gradients of all layers, from the dZ^T copies kept above
        BiasArgs b{};
        b.lddzt = mb;
        b.M = M;
        int blocks = 0;
        for (int l = 1; l <= L; ++l) {
            b.dzt[b.nseg] = n->dzT[l];
            b.db[b.nseg] = n->gb[l - 1];
            b.n[b.nseg] = n->pad[l];
            b.first[b.nseg++] = blocks;
            blocks += (n->pad[l] + 3) / 4;
        }
        b.first[b.nseg] = blocks;
        hipLaunchKernelGGL(k_mlp_bias_grad, dim3(blocks), dim3(256), 0, n->stream, b);
    }
    FK_MHIP(n, hipGetLastError());
    if (loss_host) {
        FK_MHIP(n, hipMemcpyAsync(loss_host, n->loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
        FK_MHIP(n, hipStreamSynchronize(n->stream));
    }
    return FK_OK;
}

extern "C" int fk_mlp_adamw(fk_mlp* n, double lr, double beta1, double beta2, double eps, double weight_decay,
                            int64_t step)
{
    if (!n || step < 1) return FK_E_INVALID;
    AdamArgs a{};
    a.lr = (float)lr;
    a.b1 = (float)beta1;
    a.b2 = (float)beta2;
    a.eps = (float)eps;
    a.c1 = (float)(1.0 - std::pow(beta1, (double)step));
    a.c2 = (float)(1.0 - std::pow(beta2, (double)step));
    int blocks = 0;
    for (int l = 0; l < n->L; ++l) {
        AdamSeg& w = a.seg[a.nseg];
        w.w = n->w[l];
        w.g = n->gw[l];
        w.m = n->mw[l];
        w.v = n->vw[l];
        w.wbf = n->wbf[l];
        w.wtbf = n->wtbf[l];
        w.ld = n->pad[l];
        w.ldT = n->pad[l + 1];
        w.count = n->pad[l + 1] * n->pad[l];
        w.wd = (float)weight_decay;
        a.first[a.nseg++] = blocks;
        blocks += (n->pad[l + 1] / 32) * ((n->pad[l] + 31) / 32);   // 32 x 32 tiles
        AdamSeg& b = a.seg[a.nseg];   // bias: no weight decay, no bf16 copies
        b.w = n->b[l];
        b.g = n->gb[l];
        b.m = n->mb[l];
        b.v = n->vb[l];
        b.ld = 1;
        b.ldT = 1;
        b.count = n->pad[l + 1];
        b.wd = 0.0f;
        a.first[a.nseg++] = blocks;
        blocks += (b.count + 255) / 256;
    }
    a.first[a.nseg] = blocks;
    hipLaunchKernelGGL(k_adamw, dim3(blocks), dim3(256), 0, n->stream, a);
    FK_MHIP(n, hipGetLastError());
    return FK_OK;
}

extern "C" int fk_mlp_train_step(fk_mlp* n, const float* x, const float* target, int M, double lr, double beta1,
                                 double beta2, double eps, double weight_decay, int64_t step)
{
    if (!n || !x || !target || M < 16 || M > n->max_batch || M % 16 || step < 1)
        return set_error(n ? &n->err : nullptr, FK_E_INVALID,
                         "fk_mlp_train_step: batch a multiple of 16 up to max_batch, step >= 1");
    const int L = n->L, mb = n->max_batch;
    // forward; the first layer reads the FP32 features itself (and stores
    // their bf16 copies), the output layer's epilogue forms the loss and dZ_L
    const XIn xi{x, n->dims[0], n->act[0], n->pad[0], n->actT[0], mb};
    int loss_tiles = 0;
    for (int l = 0; l < L; ++l) {
        GemmArgs g{};
        g.A = n->act[l];
        g.lda = n->pad[l];
        g.B = n->wbf[l];
        g.ldb = n->pad[l];
        g.M = M;
        g.N = n->pad[l + 1];
        g.K = n->pad[l];
        g.bias = n->b[l];
        g.out = n->z[l + 1];
        g.ldout = n->pad[l + 1];
        if (l + 1 < L) {
            g.act = n->act[l + 1];
            g.ldact = n->pad[l + 1];
            g.actT = n->actT[l + 1];
            g.ldactT = mb;
            g.epi = EPI_HIDDEN;
        } else {
            g.act = n->dz[L];
            g.ldact = n->pad[L];
            g.actT = n->dzT[L];
            g.ldactT = mb;
            g.target = target;
            g.dout = n->dims[L];
            g.gscale = (float)(2.0 / ((double)M * n->dims[L]));
            g.loss_part = n->loss_part;
            g.epi = EPI_OUTPUT_LOSS;
            int ntn = 0;
            loss_tiles = gemm_tiles(g, &ntn);
        }
        launch_gemm(n, g, nullptr, l == 0 ? &xi : nullptr);
    }
    // input gradients: dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1}), l = L .. 2 (1-based)
    for (int l = L; l >= 2; --l) {
        GemmArgs d{};
        d.A = n->dz[l];
        d.lda = n->pad[l];
        d.B = n->wtbf[l - 1];
        d.ldb = n->pad[l];
        d.M = M;
        d.N = n->pad[l - 1];
        d.K = n->pad[l];
        d.zin = n->z[l - 1];
        d.ldzin = n->pad[l - 1];
        d.act = n->dz[l - 1];
        d.ldact = n->pad[l - 1];
        d.actT = n->dzT[l - 1];
        d.ldactT = mb;
        d.epi = EPI_DGRAD;
        launch_gemm(n, d);
    }
    // weight gradients with AdamW, bias gradients with AdamW, the loss
    WgradAdamArgs a{};
    a.nl = L;
    int tiles = 0;
    for (int l = 0; l < L; ++l) {
        GemmArgs& g = a.p[l];
        g.A = n->dzT[l + 1];
        g.lda = mb;
        g.B = n->actT[l];
        g.ldb = mb;
        g.M = n->pad[l + 1];
        g.N = n->pad[l];
        g.K = M;
        g.epi = EPI_WGRAD;
        a.first[l] = tiles;
        tiles += gemm_tiles(g, &a.ntn[l]);
        AdamSeg& q = a.wseg[l];
        q.w = n->w[l];
        q.m = n->mw[l];
        q.v = n->vw[l];
        q.wbf = n->wbf[l];
        q.wtbf = n->wtbf[l];
        q.ld = n->pad[l];
        q.ldT = n->pad[l + 1];
        q.count = n->pad[l + 1] * n->pad[l];
        q.wd = (float)weight_decay;
        AdamSeg& bq = a.bseg[l];
        bq.w = n->b[l];
        bq.m = n->mb[l];
        bq.v = n->vb[l];
        bq.count = n->pad[l + 1];
        a.wgrad[l] = n->gw[l];
        a.bgrad[l] = n->gb[l];
    }
    a.first[L] = tiles;
    int bblocks = 0;
    for (int l = 0; l < L; ++l) {
        a.bfirst[l] = bblocks;
        bblocks += (n->pad[l + 1] + 3) / 4;
    }
    a.bfirst[L] = bblocks;
    a.loss_part = n->loss_part;
    a.nloss = loss_tiles;
    a.loss_scale = 1.0 / ((double)M * n->dims[L]);
    a.loss = n->loss;
    a.loss_acc = n->loss_acc;
    a.lr = (float)lr;
    a.b1 = (float)beta1;
    a.b2 = (float)beta2;
    a.eps = (float)eps;
    a.c1 = (float)(1.0 - std::pow(beta1, (double)step));
    a.c2 = (float)(1.0 - std::pow(beta2, (double)step));
    hipLaunchKernelGGL(k_mlp_wgrad_adam, dim3(tiles + bblocks + 1), dim3(256), 0, n->stream, a);
    FK_MHIP(n, hipGetLastError());
    n->last_m = M;
    return FK_OK;
}

extern "C" int fk_mlp_take_loss(fk_mlp* n, double* mean, int64_t* count)
{
    if (!n) return FK_E_INVALID;
    double acc[2] = {0.0, 0.0};
    FK_MHIP(n, hipMemcpyAsync(acc, n->loss_acc, sizeof(acc), hipMemcpyDeviceToHost, n->stream));
    FK_MHIP(n, hipMemsetAsync(n->loss_acc, 0, sizeof(acc), n->stream));
    FK_MHIP(n, hipStreamSynchronize(n->stream));
    if (mean) *mean = acc[1] > 0.0 ? acc[0] / acc[1] : 0.0;
    if (count) *count = (int64_t)acc[1];
    return FK_OK;
}

extern "C" int fk_mlp_sync(fk_mlp* n)
{
    if (!n) return FK_E_INVALID;
    FK_MHIP(n, hipStreamSynchronize(n->stream));
    return FK_OK;
}
