// mlp.hip -- the learned regime indicator: feature construction, the
// 192 -> 64 -> 64 -> 1 ReLU network on BF16 matrix cores (FP32 accumulation),
// its backward pass, a deterministic gradient reduction and Adam.
//
// The network predicts, from the macroscopic state at the start of a step,
// whether the plain criterion of Sec. 3.1.2 marks a cell kinetic at any of
// the next K steps (the engine runs the plain criterion every K steps as the
// fallback and the judge of the prediction).  Features of cell c, over its
// periodic 5 x 5 stencil (k = 5 (dj + 2) + (di + 2)), for stencil cell s:
//   x[7k+0] = rho_s / rho_c - 1, x[7k+1] = ux_s - ux_c, x[7k+2] = uy_s - uy_c,
//   x[7k+3] = T_s / T_c - 1, x[7k+4] = eps_s / (eps_s + 0.01),
//   x[7k+5] = A_s / (A_s + 1e-4), A = eps^2 |grad u|^2,
//   x[7k+6] = B_s / (B_s + 1e-4), B = eps^2 |grad T|^2 / T,
//   x[175] = previous mask of c, x[176..191] = 0;
// central differences, every feature a fixed order of correctly rounded FP64
// + - * / (no contraction in this file), rounded FP32 -> BF16 (nearest even).
//
// Matrix products use v_mfma_f32_16x16x16_bf16 on 64-row tiles of samples.
// The backward products take FP32 gradient matrices split into BF16 hi + lo
// parts, so that each product of a BF16 matrix with an FP32 one is carried to
// about 2^-17 relative.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>

#include "../../include/esbgk.h"
#include "device.h"

#pragma clang fp contract(off)

namespace esbgk {
namespace mlp {

constexpr int NF = 176, NIN = 192, NH = 64, ROWS = 64;
constexpr int NPARAM = NIN * NH + NH + NH * NH + NH + NH + 1;
// offsets of the flat parameter vector
constexpr int O_W1 = 0, O_B1 = O_W1 + NIN * NH, O_W2 = O_B1 + NH, O_B2 = O_W2 + NH * NH, O_W3 = O_B2 + NH,
              O_B3 = O_W3 + NH;
// LDS row strides (bf16 elements), padded against bank conflicts
constexpr int SX = NIN + 8, SH = NH + 8;

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// --------------------------------------------------------------- features

__device__ inline int wrapm(int i, int n) { i %= n; return i < 0 ? i + n : i; }

// e, gA, gB of cell c from the fields ux, uy, T, eps (idx2 = 2 dx, idy2 = 2 dy).
__device__ inline void derived_cell(int nx, int ny, double idx2, double idy2, const double *ux, const double *uy,
                                    const double *T, const double *eps, int c, double out[3]) {
    const int i = c % nx, j = c / nx;
    const size_t ce = (size_t)j * nx + wrapm(i + 1, nx), cw = (size_t)j * nx + wrapm(i - 1, nx);
    const size_t cn = (size_t)wrapm(j + 1, ny) * nx + i, cs = (size_t)wrapm(j - 1, ny) * nx + i;
    // (q_{i+1} - q_{i-1}) / (2 dx)
    const double uxx = (ux[ce] - ux[cw]) / idx2, uxy = (ux[cn] - ux[cs]) / idy2;
    const double uyx = (uy[ce] - uy[cw]) / idx2, uyy = (uy[cn] - uy[cs]) / idy2;
    const double Tx = (T[ce] - T[cw]) / idx2, Ty = (T[cn] - T[cs]) / idy2;
    const double gu2 = ((uxx * uxx + uxy * uxy) + uyx * uyx) + uyy * uyy;
    const double gT2 = Tx * Tx + Ty * Ty;
    const double e = eps[c];
    const double e2 = e * e;
    const double A = e2 * gu2;
    const double B = (e2 * gT2) / T[c];
    out[0] = e / (e + 0.01);
    out[1] = A / (A + 1e-4);
    out[2] = B / (B + 1e-4);
}

// Per-cell e, gA, gB of every snapshot: derived[s][3][nc].
__global__ void derived_kernel(int nx, int ny, double idx2, double idy2, const double *fields, int nsnap,
                               double *derived) {
    const size_t nc = (size_t)nx * ny;
    const size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (t >= nc * nsnap) return;
    const size_t snap = t / nc;
    const int c = (int)(t % nc);
    const double *F = fields + snap * 6 * nc;
    double o[3];
    derived_cell(nx, ny, idx2, idy2, F + nc, F + 2 * nc, F + 3 * nc, F + 4 * nc, c, o);
    double *D = derived + snap * 3 * nc;
    D[c] = o[0];
    D[nc + c] = o[1];
    D[2 * nc + c] = o[2];
}

// The 7 features of stencil index k (0..24) of cell c (BF16 bits).
__device__ inline void stencil_features(int nx, int ny, const double *rho, const double *ux, const double *uy,
                                        const double *T, const double *D, size_t nc, int c, int k, double rc,
                                        double uxc, double uyc, double Tc, uint16_t out[7]) {
    const int i = c % nx, j = c / nx;
    const int dj = k / 5 - 2, di = k % 5 - 2;
    const size_t s = (size_t)wrapm(j + dj, ny) * nx + wrapm(i + di, nx);
    const double v[7] = {rho[s] / rc - 1.0, ux[s] - uxc, uy[s] - uyc, T[s] / Tc - 1.0, D[s], D[nc + s], D[2 * nc + s]};
#pragma unroll
    for (int m = 0; m < 7; ++m) out[m] = bf16_bits((float)v[m]);
}

// X[n][192] (BF16 bits) of the samples (snapshot, cell).
// Samples outside [0, nsnap) x [0, nc) get a zero row.
__global__ void features_kernel(int nx, int ny, const double *fields, const double *derived, int nsnap,
                                const int *samples, int n, uint16_t *X) {
    const int r = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (r >= n) return;
    const size_t nc = (size_t)nx * ny;
    const int sn = samples[2 * r];
    const int c = samples[2 * r + 1];
    uint16_t *row = X + (size_t)r * NIN;
    if (sn < 0 || sn >= nsnap || c < 0 || (size_t)c >= nc) {
        for (int m = 0; m < NIN; ++m) row[m] = 0;
        return;
    }
    const size_t snap = (size_t)sn;
    const double *F = fields + snap * 6 * nc;
    const double *D = derived + snap * 3 * nc;
    const double rc = F[c], uxc = F[nc + c], uyc = F[2 * nc + c], Tc = F[3 * nc + c];
    for (int k = 0; k < 25; ++k) {
        uint16_t o[7];
        stencil_features(nx, ny, F, F + nc, F + 2 * nc, F + 3 * nc, D, nc, c, k, rc, uxc, uyc, Tc, o);
#pragma unroll
        for (int m = 0; m < 7; ++m) row[7 * k + m] = o[m];
    }
    row[175] = bf16_bits((float)F[5 * nc + c]);
    for (int m = NF; m < NIN; ++m) row[m] = 0;
}

// --------------------------------------------------------------- weights

struct Net {
    float *p;            // FP32 master parameters, flat (W1 [192][64] by input, b1, W2 [64][64], b2, w3, b3)
    float *m, *v;        // Adam moments
    uint16_t *w1t;       // BF16 W1 transposed [64][192]
    uint16_t *w2t;       // BF16 W2 transposed [64][64]  (B operand of the forward product)
    uint16_t *w2n;       // BF16 W2 [64][64] by input     (B operand of dH1 = dZ2 W2^T)
    uint16_t *w3;        // BF16 w3 [64]
    float *partial;      // per-block gradient partials [max_blocks][NPARAM]
    float *grad;         // reduced gradient [NPARAM]
    float *lpart;        // per-block loss partials [max_blocks]
    int max_blocks;
};

__global__ void prepare_kernel(Net net) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < NIN * NH) {
        const int k = t / NH, n = t % NH;  // W1[k][n]
        net.w1t[n * NIN + k] = bf16_bits(net.p[O_W1 + t]);
    }
    if (t < NH * NH) {
        const int k = t / NH, n = t % NH;  // W2[k][n]
        const uint16_t b = bf16_bits(net.p[O_W2 + t]);
        net.w2t[n * NH + k] = b;
        net.w2n[t] = b;
    }
    if (t < NH) net.w3[t] = bf16_bits(net.p[O_W3 + t]);
}

// ------------------------------------------------------------ MFMA tiles
//
// v_mfma_f32_16x16x16_bf16, wave64; with r = lane % 16, g = lane / 16:
//   A operand: A[r][4g + j],  B operand: B[4g + j][r],  result: D[4g + j][r].
// Operands come from LDS with k contiguous: A as [m][k], B as Bt = [n][k].

__device__ inline v4f mfma(v4s a, v4s b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

__device__ inline v4s lds4(const uint16_t *p) {
    const uint2 u = *reinterpret_cast<const uint2 *>(p);
    v4s r;
    r[0] = (short)(u.x & 0xFFFF); r[1] = (short)(u.x >> 16);
    r[2] = (short)(u.y & 0xFFFF); r[3] = (short)(u.y >> 16);
    return r;
}

// Accumulate the 16 x 16 tile (tm, tn) of A Bt^T over K into acc.
__device__ inline v4f tile_mm(v4f acc, const uint16_t *A, int lda, const uint16_t *Bt, int ldb, int tm, int tn,
                              int K, int lane) {
    const int r = lane & 15, g = lane >> 4;
    const uint16_t *a = A + (size_t)(tm * 16 + r) * lda + 4 * g;
    const uint16_t *b = Bt + (size_t)(tn * 16 + r) * ldb + 4 * g;
    for (int kk = 0; kk < K; kk += 16) acc = mfma(lds4(a + kk), lds4(b + kk), acc);
    return acc;
}

// Same with A read with a stride along k (A[m][k] = src[k * ldk + m]): the
// transposed feature tile of dW1 = X^T dZ1.
__device__ inline v4f tile_mm_at(v4f acc, const uint16_t *src, int ldk, const uint16_t *Bt, int ldb, int tm, int tn,
                                 int K, int lane) {
    const int r = lane & 15, g = lane >> 4;
    const uint16_t *b = Bt + (size_t)(tn * 16 + r) * ldb + 4 * g;
    for (int kk = 0; kk < K; kk += 16) {
        v4s a;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) a[jj] = (short)src[(size_t)(kk + 4 * g + jj) * ldk + tm * 16 + r];
        acc = mfma(a, lds4(b + kk), acc);
    }
    return acc;
}

// ------------------------------------------------------------ forward

// Shared-memory image of one 64-row tile and the weights it needs.
struct FwdLds {
    uint16_t x[ROWS][SX];
    uint16_t w1t[NH][SX];
    uint16_t w2t[NH][SH];
    uint16_t h1[ROWS][SH];
    uint16_t h2[ROWS][SH];
    float w3[NH], b1[NH], b2[NH];
};

__device__ inline void load_weights_fwd(FwdLds &L, const Net &net, int tid, int nthr) {
    for (int t = tid; t < NH * NIN / 4; t += nthr) {
        const int n = t / (NIN / 4), k4 = t % (NIN / 4);
        *reinterpret_cast<uint2 *>(&L.w1t[n][4 * k4]) = *reinterpret_cast<const uint2 *>(net.w1t + n * NIN + 4 * k4);
    }
    for (int t = tid; t < NH * NH / 4; t += nthr) {
        const int n = t / (NH / 4), k4 = t % (NH / 4);
        *reinterpret_cast<uint2 *>(&L.w2t[n][4 * k4]) = *reinterpret_cast<const uint2 *>(net.w2t + n * NH + 4 * k4);
    }
    for (int t = tid; t < NH; t += nthr) {
        L.w3[t] = bf16_val(net.w3[t]);
        L.b1[t] = net.p[O_B1 + t];
        L.b2[t] = net.p[O_B2 + t];
    }
}

__device__ inline void load_x_tile(FwdLds &L, const uint16_t *X, int row0, int n, int tid, int nthr) {
    for (int t = tid; t < ROWS * NIN / 4; t += nthr) {
        const int r = t / (NIN / 4), k4 = t % (NIN / 4);
        uint2 v = make_uint2(0u, 0u);
        if (row0 + r < n) v = *reinterpret_cast<const uint2 *>(X + (size_t)(row0 + r) * NIN + 4 * k4);
        *reinterpret_cast<uint2 *>(&L.x[r][4 * k4]) = v;
    }
}

// Forward of the tile in L.x: h1, h2 (BF16) in LDS; returns the logit of
// row tid / 4 in every lane of its quad (threads 0..255).
__device__ inline float forward_tile(FwdLds &L, float b3, int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    // layer 1: wave w owns rows 16 w .. 16 w + 15, all 64 units
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) {
        v4f acc = {0, 0, 0, 0};
        acc = tile_mm(acc, &L.x[0][0], SX, &L.w1t[0][0], SX, wave, tn, NIN, lane);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int row = wave * 16 + 4 * g + jj, col = tn * 16 + r;
            L.h1[row][col] = bf16_bits(fmaxf(acc[jj] + L.b1[col], 0.0f));
        }
    }
    __syncthreads();
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) {
        v4f acc = {0, 0, 0, 0};
        acc = tile_mm(acc, &L.h1[0][0], SH, &L.w2t[0][0], SH, wave, tn, NH, lane);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int row = wave * 16 + 4 * g + jj, col = tn * 16 + r;
            L.h2[row][col] = bf16_bits(fmaxf(acc[jj] + L.b2[col], 0.0f));
        }
    }
    __syncthreads();
    // logit: 4 lanes per row, 16 units each, then a quad butterfly
    const int row = tid >> 2, part = tid & 3;
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += bf16_val(L.h2[row][16 * part + k]) * L.w3[16 * part + k];
    s += partner<0>(s);
    s += partner<1>(s);
    return s + b3;
}

__global__ __launch_bounds__(256) void forward_kernel(Net net, const uint16_t *X, int n, float *logits) {
    __shared__ FwdLds L;
    const int tid = (int)threadIdx.x;
    load_weights_fwd(L, net, tid, 256);
    const float b3 = net.p[O_B3];
    const int ntiles = (n + ROWS - 1) / ROWS;
    for (int tile = (int)blockIdx.x; tile < ntiles; tile += (int)gridDim.x) {
        __syncthreads();
        load_x_tile(L, X, tile * ROWS, n, tid, 256);
        __syncthreads();
        const float z = forward_tile(L, b3, tid);
        const int row = tile * ROWS + (tid >> 2);
        if ((tid & 3) == 0 && row < n) logits[row] = z;
    }
}

// Derived fields of the engine's current state: prim SoA [4][nc], eps [nc].
__global__ void grid_derived_kernel(int nx, int ny, double idx2, double idy2, const double *prim, const double *eps,
                                    double *derived) {
    const size_t nc = (size_t)nx * ny;
    const int c = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if ((size_t)c >= nc) return;
    double o[3];
    derived_cell(nx, ny, idx2, idy2, prim + nc, prim + 2 * nc, prim + 3 * nc, eps, c, o);
    derived[c] = o[0];
    derived[nc + c] = o[1];
    derived[2 * nc + c] = o[2];
}

// Inference over the whole grid for the engine's check step: each 64-cell
// tile's features are formed in LDS (4 threads per cell; the same operations
// as features_kernel), the network runs on them, and the mask of the next
// steps is written directly: out = plain | (logit > threshold).  Counts the
// judge counters against the mask in use (when counters is given).
__global__ __launch_bounds__(256) void grid_mask_kernel(Net net, int nx, int ny, const double *prim, const double *eps,
                                                        const uint8_t *in_use, const double *derived,
                                                        const uint8_t *plain, float threshold, uint8_t *out,
                                                        long long *counters) {
    __shared__ FwdLds L;
    const int tid = (int)threadIdx.x, row = tid >> 2, part = tid & 3;
    load_weights_fwd(L, net, tid, 256);
    const float b3 = net.p[O_B3];
    const size_t nc = (size_t)nx * ny;
    const int ntiles = (int)((nc + ROWS - 1) / ROWS);
    const double *rho = prim, *ux = prim + nc, *uy = prim + 2 * nc, *T = prim + 3 * nc;
    int cnt[3] = {0, 0, 0};
    for (int tile = (int)blockIdx.x; tile < ntiles; tile += (int)gridDim.x) {
        __syncthreads();
        const int c = tile * ROWS + row;
        if ((size_t)c < nc) {
            const double rc = rho[c], uxc = ux[c], uyc = uy[c], Tc = T[c];
            for (int k = part; k < 25; k += 4) {
                uint16_t o[7];
                stencil_features(nx, ny, rho, ux, uy, T, derived, nc, c, k, rc, uxc, uyc, Tc, o);
#pragma unroll
                for (int m = 0; m < 7; ++m) L.x[row][7 * k + m] = o[m];
            }
            if (part == 0) L.x[row][175] = bf16_bits(in_use[c] ? 1.0f : 0.0f);
        } else {
            for (int k = part; k < 25; k += 4)
#pragma unroll
                for (int m = 0; m < 7; ++m) L.x[row][7 * k + m] = 0;
            if (part == 0) L.x[row][175] = 0;
        }
        for (int m = NF + part; m < NIN; m += 4) L.x[row][m] = 0;
        __syncthreads();
        const float z = forward_tile(L, b3, tid);
        if (part == 0 && (size_t)c < nc) {
            const bool p = plain[c], u = in_use[c];
            out[c] = (uint8_t)(p || z > threshold);
            cnt[0] += p && !u;
            cnt[1] += u && !p;
            cnt[2] += p;
        }
    }
    if (counters) {
        __shared__ int red[3];
        if (tid < 3) red[tid] = 0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q)
            if (cnt[q]) atomicAdd(&red[q], cnt[q]);
        __syncthreads();
        if (tid < 3 && red[tid]) atomicAdd((unsigned long long *)&counters[1 + tid], (unsigned long long)red[tid]);
        if (tid == 0 && blockIdx.x == 0) atomicAdd((unsigned long long *)&counters[0], 1ull);
    }
}

// ------------------------------------------------------------ backward

struct BwdLds {
    FwdLds f;
    uint16_t w2n[NH][SH];
    uint16_t h1t[NH][SH];     // H1^T [unit][row]
    uint16_t dz2[2][ROWS][SH];  // dZ2 hi / lo [row][unit]
    uint16_t dz2t[2][NH][SH];   // dZ2^T hi / lo [unit][row]
    uint16_t dz1t[2][NH][SH];   // dZ1^T hi / lo [unit][row]
    float dz[ROWS];
};

__device__ inline void split(float v, uint16_t &hi, uint16_t &lo) {
    hi = bf16_bits(v);
    lo = bf16_bits(v - bf16_val(hi));
}

// One 64-row tile per block: forward, logistic-loss gradient, backward;
// writes the tile's gradient partials and loss partial (sum over its rows of
// the per-row loss, divided by n).
__global__ __launch_bounds__(256) void train_tile_kernel(Net net, const uint16_t *X, const float *y, int n,
                                                         float wpos) {
    extern __shared__ __align__(16) unsigned char smem[];
    BwdLds &L = *reinterpret_cast<BwdLds *>(smem);
    const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int tile = (int)blockIdx.x, row0 = tile * ROWS;
    load_weights_fwd(L.f, net, tid, 256);
    for (int t = tid; t < NH * NH / 4; t += 256) {
        const int k = t / (NH / 4), n4 = t % (NH / 4);
        *reinterpret_cast<uint2 *>(&L.w2n[k][4 * n4]) = *reinterpret_cast<const uint2 *>(net.w2n + k * NH + 4 * n4);
    }
    load_x_tile(L.f, X, row0, n, tid, 256);
    __syncthreads();
    const float z = forward_tile(L.f, net.p[O_B3], tid);
    float *part = net.partial + (size_t)tile * NPARAM;
    // dz = (sigma(z) (wpos y + 1 - y) - wpos y) / n, zero on padding rows
    {
        const int row = tid >> 2;
        const bool valid = row0 + row < n;
        const float yy = valid ? y[row0 + row] : 0.0f;
        const float sg = 1.0f / (1.0f + __expf(-z));
        const float d = valid ? (sg * (wpos * yy + 1.0f - yy) - wpos * yy) / (float)n : 0.0f;
        // per-row loss: wpos y softplus(-z) + (1 - y) softplus(z)
        const float sp_pos = log1pf(__expf(-fabsf(z))) + fmaxf(z, 0.0f);   // softplus(z)
        const float sp_neg = sp_pos - z;                                    // softplus(-z)
        float lrow = valid ? (wpos * yy * sp_neg + (1.0f - yy) * sp_pos) / (float)n : 0.0f;
        if ((tid & 3) == 0) L.dz[row] = d;
        // loss partial of the tile: rows summed in a fixed tree
        lrow = (tid & 3) == 0 ? lrow : 0.0f;
        lrow += partner<0>(lrow); lrow += partner<1>(lrow); lrow += partner<2>(lrow);
        lrow += partner<3>(lrow); lrow += partner<4>(lrow);
        lrow = readlane(lrow, 0) + readlane(lrow, 32);
        __shared__ float lw[4];
        if (lane == 0) lw[wave] = lrow;
        // H1^T for dW2
        for (int t = tid; t < ROWS * NH; t += 256) {
            const int rr = t / NH, u = t % NH;
            L.h1t[u][rr] = L.f.h1[rr][u];
        }
        __syncthreads();
        if (tid == 0) net.lpart[tile] = (lw[0] + lw[1]) + (lw[2] + lw[3]);
    }
    // dw3, db3, dZ2, db2: thread u < 64 owns unit u
    if (tid < NH) {
        const int u = tid;
        float s3 = 0.0f, s2 = 0.0f;
        for (int rr = 0; rr < ROWS; ++rr) {
            const float h2 = bf16_val(L.f.h2[rr][u]);
            s3 += h2 * L.dz[rr];
            const float d2 = h2 > 0.0f ? L.dz[rr] * L.f.w3[u] : 0.0f;
            s2 += d2;
            uint16_t hi, lo;
            split(d2, hi, lo);
            L.dz2[0][rr][u] = hi; L.dz2[1][rr][u] = lo;
            L.dz2t[0][u][rr] = hi; L.dz2t[1][u][rr] = lo;
        }
        part[O_W3 + u] = s3;
        part[O_B2 + u] = s2;
    }
    if (tid == NH) {
        float s = 0.0f;
        for (int rr = 0; rr < ROWS; ++rr) s += L.dz[rr];
        part[O_B3] = s;
    }
    __syncthreads();
    // dW2 = H1^T dZ2 (64 x 64) and dH1 = dZ2 W2^T (64 x 64): wave w owns row strip w
#pragma unroll
    for (int tn = 0; tn < 4; ++tn) {
        v4f acc = {0, 0, 0, 0};
        acc = tile_mm(acc, &L.h1t[0][0], SH, &L.dz2t[0][0][0], SH, wave, tn, ROWS, lane);
        acc = tile_mm(acc, &L.h1t[0][0], SH, &L.dz2t[1][0][0], SH, wave, tn, ROWS, lane);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int k = wave * 16 + 4 * g + jj, nn = tn * 16 + r;  // W2[k][nn]
            part[O_W2 + k * NH + nn] = acc[jj];
        }
        v4f dh = {0, 0, 0, 0};
        dh = tile_mm(dh, &L.dz2[0][0][0], SH, &L.w2n[0][0], SH, wave, tn, NH, lane);
        dh = tile_mm(dh, &L.dz2[1][0][0], SH, &L.w2n[0][0], SH, wave, tn, NH, lane);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int rr = wave * 16 + 4 * g + jj, u = tn * 16 + r;
            const float d1 = bf16_val(L.f.h1[rr][u]) > 0.0f ? dh[jj] : 0.0f;
            uint16_t hi, lo;
            split(d1, hi, lo);
            L.dz1t[0][u][rr] = hi; L.dz1t[1][u][rr] = lo;
        }
    }
    __syncthreads();
    // db1: thread u < 64 sums its column of dZ1 (hi + lo, the value the product uses)
    if (tid < NH) {
        float s = 0.0f;
        for (int rr = 0; rr < ROWS; ++rr) s += bf16_val(L.dz1t[0][tid][rr]) + bf16_val(L.dz1t[1][tid][rr]);
        part[O_B1 + tid] = s;
    }
    // dW1 = X^T dZ1 (192 x 64): 12 x 4 tiles, 12 per wave
    for (int t = wave; t < 48; t += 4) {
        const int tm = t / 4, tn = t % 4;
        v4f acc = {0, 0, 0, 0};
        acc = tile_mm_at(acc, &L.f.x[0][0], SX, &L.dz1t[0][0][0], SH, tm, tn, ROWS, lane);
        acc = tile_mm_at(acc, &L.f.x[0][0], SX, &L.dz1t[1][0][0], SH, tm, tn, ROWS, lane);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int k = tm * 16 + 4 * g + jj, nn = tn * 16 + r;  // W1[k][nn]
            part[O_W1 + k * NH + nn] = acc[jj];
        }
    }
}

// grad[p] = sum over tiles of partial[tile][p] (tile order fixed); loss too.
__global__ void reduce_kernel(Net net, int ntiles, float *loss) {
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p < NPARAM) {
        float s = 0.0f;
        for (int t = 0; t < ntiles; ++t) s += net.partial[(size_t)t * NPARAM + p];
        net.grad[p] = s;
    }
    if (p == 0 && loss) {
        float s = 0.0f;
        for (int t = 0; t < ntiles; ++t) s += net.lpart[t];
        *loss = s;
    }
}

// Bias-corrected Adam (Kingma & Ba, 2015) on the FP32 master parameters.
__global__ void adam_kernel(Net net, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= NPARAM) return;
    if (p >= O_W1 + NF * NH && p < O_B1) return;  // weights of the zero padding inputs stay 0
    const float gr = net.grad[p];
    const float m = b1 * net.m[p] + (1.0f - b1) * gr;
    const float v = b2 * net.v[p] + (1.0f - b2) * gr * gr;
    net.m[p] = m;
    net.v[p] = v;
    net.p[p] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

__global__ void zero_kernel(float *a, int n) {
    const int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (t < n) a[t] = 0.0f;
}

}  // namespace mlp
}  // namespace esbgk

// ------------------------------------------------------------------ C ABI

using namespace esbgk::mlp;

struct esbgk_mlp {
    Net net{};
    int max_batch = 0;
    long long t = 0;  // Adam step count
};

namespace {

thread_local char g_mlp_err[256] = "";

int mfail(int code, const char *msg) {
    snprintf(g_mlp_err, sizeof g_mlp_err, "%s", msg);
    return code;
}

#define MCHK(x)                                                                       \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) return mfail(ESBGK_EDEVICE, hipGetErrorString(e_));   \
    } while (0)

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

struct MlpLayout {
    size_t p, m, v, w1t, w2t, w2n, w3, partial, grad, lpart, total;
};

MlpLayout mlp_layout(int max_batch) {
    MlpLayout L;
    const size_t tiles = (size_t)(max_batch + ROWS - 1) / ROWS;
    size_t off = 0;
    auto take = [&](size_t b) { size_t o = off; off += a256(b); return o; };
    L.p = take(NPARAM * 4); L.m = take(NPARAM * 4); L.v = take(NPARAM * 4);
    L.w1t = take(NIN * NH * 2); L.w2t = take(NH * NH * 2); L.w2n = take(NH * NH * 2); L.w3 = take(NH * 2);
    L.partial = take(tiles * NPARAM * 4); L.grad = take(NPARAM * 4); L.lpart = take(tiles * 4);
    L.total = off;
    return L;
}

hipStream_t S(void *s) { return (hipStream_t)s; }

int prepare(esbgk_mlp *m, hipStream_t st) {
    hipLaunchKernelGGL(prepare_kernel, dim3((NIN * NH + 255) / 256), dim3(256), 0, st, m->net);
    MCHK(hipGetLastError());
    return ESBGK_OK;
}

int check_batch(const esbgk_mlp *m, int n) {
    if (!m) return mfail(ESBGK_EINVAL, "null network");
    if (n < 1 || n > m->max_batch) return mfail(ESBGK_EINVAL, "batch size outside [1, max_batch]");
    return ESBGK_OK;
}

int train_tiles(esbgk_mlp *m, const uint16_t *X, const float *y, int n, float wpos, float *loss, hipStream_t st) {
    const int tiles = (n + ROWS - 1) / ROWS;
    const size_t lds = sizeof(BwdLds);
    hipLaunchKernelGGL(train_tile_kernel, dim3(tiles), dim3(256), lds, st, m->net, X, y, n, wpos);
    MCHK(hipGetLastError());
    hipLaunchKernelGGL(reduce_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, m->net, tiles, loss);
    MCHK(hipGetLastError());
    return ESBGK_OK;
}

}  // namespace

namespace esbgk {

// Check-step inference of the engine (see grid_mask_kernel): derived fields
// into `derived` (3 nc doubles), then the mask of the next steps.
hipError_t launch_learned_mask(esbgk_mlp *m, int nx, int ny, double lx, double ly, const double *prim,
                               const double *eps, const uint8_t *in_use, double *derived, const uint8_t *plain,
                               float threshold, uint8_t *out, long long *counters, hipStream_t st) {
    const int nc = nx * ny;
    hipLaunchKernelGGL(grid_derived_kernel, dim3((nc + 255) / 256), dim3(256), 0, st, nx, ny, 2.0 * (lx / nx),
                       2.0 * (ly / ny), prim, eps, derived);
    const int tiles = (nc + ROWS - 1) / ROWS;
    hipLaunchKernelGGL(grid_mask_kernel, dim3((unsigned)std::min(tiles, 4096)), dim3(256), 0, st, m->net, nx, ny, prim,
                       eps, in_use, derived, plain, threshold, out, counters);
    return hipGetLastError();
}

}  // namespace esbgk

extern "C" {

const char *esbgk_mlp_last_error(void) { return g_mlp_err; }

int esbgk_mlp_param_count(void) { return NPARAM; }

int esbgk_mlp_workspace_size(int max_batch, size_t *bytes) {
    if (max_batch < 1 || !bytes) return mfail(ESBGK_EINVAL, "max_batch < 1 or null output");
    *bytes = mlp_layout(max_batch).total;
    return ESBGK_OK;
}

int esbgk_mlp_create(int max_batch, void *d_workspace, size_t bytes, esbgk_mlp **out) {
    if (!out) return mfail(ESBGK_EINVAL, "null output");
    *out = nullptr;
    if (max_batch < 1) return mfail(ESBGK_EINVAL, "max_batch < 1");
    if (!d_workspace || ((uintptr_t)d_workspace & 255)) return mfail(ESBGK_EINVAL, "workspace null or not 256-byte aligned");
    const MlpLayout L = mlp_layout(max_batch);
    if (bytes < L.total) return mfail(ESBGK_ENOMEM, "workspace too small");
    static_assert(sizeof(BwdLds) <= 160 * 1024, "training tile exceeds LDS");
    hipError_t e = hipFuncSetAttribute((const void *)train_tile_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)sizeof(BwdLds));
    if (e != hipSuccess) return mfail(ESBGK_EDEVICE, hipGetErrorString(e));
    esbgk_mlp *m = new (std::nothrow) esbgk_mlp;
    if (!m) return mfail(ESBGK_ENOMEM, "host allocation failed");
    char *w = (char *)d_workspace;
    m->net.p = (float *)(w + L.p); m->net.m = (float *)(w + L.m); m->net.v = (float *)(w + L.v);
    m->net.w1t = (uint16_t *)(w + L.w1t); m->net.w2t = (uint16_t *)(w + L.w2t); m->net.w2n = (uint16_t *)(w + L.w2n);
    m->net.w3 = (uint16_t *)(w + L.w3);
    m->net.partial = (float *)(w + L.partial); m->net.grad = (float *)(w + L.grad); m->net.lpart = (float *)(w + L.lpart);
    m->net.max_blocks = (max_batch + ROWS - 1) / ROWS;
    m->max_batch = max_batch;
    *out = m;
    return ESBGK_OK;
}

void esbgk_mlp_destroy(esbgk_mlp *m) { delete m; }

int esbgk_mlp_set_weights(esbgk_mlp *m, const float *d_params, void *stream) {
    if (!m || !d_params) return mfail(ESBGK_EINVAL, "null argument");
    hipStream_t st = S(stream);
    MCHK(hipMemcpyAsync(m->net.p, d_params, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(zero_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, m->net.m, NPARAM);
    hipLaunchKernelGGL(zero_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, m->net.v, NPARAM);
    MCHK(hipGetLastError());
    m->t = 0;
    return prepare(m, st);
}

int esbgk_mlp_get_weights(esbgk_mlp *m, float *d_params, void *stream) {
    if (!m || !d_params) return mfail(ESBGK_EINVAL, "null argument");
    MCHK(hipMemcpyAsync(d_params, m->net.p, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, S(stream)));
    return ESBGK_OK;
}

int esbgk_mlp_derived(int nx, int ny, double lx, double ly, const double *d_fields, int nsnap, double *d_derived,
                      void *stream) {
    if (nx < 1 || ny < 1 || nsnap < 1 || !d_fields || !d_derived || !(lx > 0) || !(ly > 0))
        return mfail(ESBGK_EINVAL, "bad grid or null pointer");
    const size_t tot = (size_t)nx * ny * nsnap;
    hipLaunchKernelGGL(derived_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, S(stream), nx, ny,
                       2.0 * (lx / nx), 2.0 * (ly / ny), d_fields, nsnap, d_derived);
    MCHK(hipGetLastError());
    return ESBGK_OK;
}

int esbgk_mlp_features(int nx, int ny, const double *d_fields, const double *d_derived, int nsnap,
                       const int *d_samples, int n, uint16_t *d_X, void *stream) {
    if (nx < 1 || ny < 1 || nsnap < 1 || n < 0 || !d_fields || !d_derived || (n > 0 && (!d_samples || !d_X)))
        return mfail(ESBGK_EINVAL, "bad grid or null pointer");
    if (n == 0) return ESBGK_OK;
    hipLaunchKernelGGL(features_kernel, dim3((n + 255) / 256), dim3(256), 0, S(stream), nx, ny, d_fields, d_derived,
                       nsnap, d_samples, n, d_X);
    MCHK(hipGetLastError());
    return ESBGK_OK;
}

int esbgk_mlp_forward(esbgk_mlp *m, const uint16_t *d_X, int n, float *d_logits, void *stream) {
    if (!m) return mfail(ESBGK_EINVAL, "null network");
    if (n < 0 || (n > 0 && (!d_X || !d_logits))) return mfail(ESBGK_EINVAL, "bad batch or null pointer");
    if (n == 0) return ESBGK_OK;
    const int tiles = (n + ROWS - 1) / ROWS;
    hipLaunchKernelGGL(forward_kernel, dim3((unsigned)std::min(tiles, 2048)), dim3(256), 0, S(stream), m->net, d_X, n,
                       d_logits);
    MCHK(hipGetLastError());
    return ESBGK_OK;
}

int esbgk_mlp_gradients(esbgk_mlp *m, const uint16_t *d_X, const float *d_y, int n, float wpos, float *d_grad,
                        float *d_loss, void *stream) {
    int rc = check_batch(m, n);
    if (rc) return rc;
    if (!d_X || !d_y || !d_grad) return mfail(ESBGK_EINVAL, "null pointer");
    hipStream_t st = S(stream);
    if ((rc = train_tiles(m, d_X, d_y, n, wpos, d_loss, st))) return rc;
    MCHK(hipMemcpyAsync(d_grad, m->net.grad, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, st));
    return ESBGK_OK;
}

int esbgk_mlp_train_step(esbgk_mlp *m, const uint16_t *d_X, const float *d_y, int n, float wpos, float lr,
                         float *d_loss, void *stream) {
    int rc = check_batch(m, n);
    if (rc) return rc;
    if (!d_X || !d_y || !(lr > 0.0f)) return mfail(ESBGK_EINVAL, "null pointer or lr <= 0");
    hipStream_t st = S(stream);
    if ((rc = train_tiles(m, d_X, d_y, n, wpos, d_loss, st))) return rc;
    m->t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, (double)m->t)), c2 = (float)(1.0 - std::pow(b2, (double)m->t));
    hipLaunchKernelGGL(adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, m->net, lr, (float)b1, (float)b2,
                       1e-8f, c1, c2);
    MCHK(hipGetLastError());
    return prepare(m, st);
}

}  // extern "C"
