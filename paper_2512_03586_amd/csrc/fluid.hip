// fluid.hip -- per-cell kernels: the Euler finite-volume stage on fluid cells,
// primitive/conserved conversions, the regime indicator, cell classification
// and the deterministic stream compaction of kinetic / buffer cells.
#include "kernels.h"

namespace esbgk {

__device__ inline int wrapc(int i, int n) { i %= n; return i < 0 ? i + n : i; }

// ------------------------------------------------------------------ Euler

__device__ inline double dminmod(double a, double b) {
    if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return 0.0;
    return a > 0.0 ? fmin(a, b) : fmax(a, b);
}

// Physical flux of the compressible Euler system in direction d
// (eq. Euler_Compact, gamma = 2 so P = E - rho|u|^2/2).
__device__ inline void euler_flux(const double U[4], int d, double F[4], double *speed) {
    const double rho = U[0], irho = 1.0 / rho, ux = U[1] * irho, uy = U[2] * irho, E = U[3];
    const double P = E - 0.5 * rho * (ux * ux + uy * uy);
    const double un = d == 0 ? ux : uy;
    F[0] = rho * un;
    F[1] = U[1] * un + (d == 0 ? P : 0.0);
    F[2] = U[2] * un + (d == 1 ? P : 0.0);
    F[3] = un * (E + P);
    *speed = fabs(un) + sqrt(2.0 * P * irho);
}

// Rusanov flux (Sec. 3.2, Lax-Friedrichs type) at the face between stencil
// cells 1 and 2 of st[q][0..3] (the 4 cells along direction d), with the
// kinetic transport's reconstruction applied component-wise to U.
__device__ inline void euler_face_vals(const double st[4][4], int d, int recon, double Fh[4]) {
    double UL[4], UR[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double a = st[q][0], b = st[q][1], e = st[q][2], g = st[q][3];
        double sp = 0.0, sq = 0.0;
        if (recon == 1) {
            sp = dminmod(b - a, e - b);
            sq = dminmod(e - b, g - e);
        }
        UL[q] = b + 0.5 * sp;
        UR[q] = e - 0.5 * sq;
    }
    double FL[4], FR[4], aL, aR;
    euler_flux(UL, d, FL, &aL);
    euler_flux(UR, d, FR, &aR);
    const double s = fmax(aL, aR);
#pragma unroll
    for (int q = 0; q < 4; ++q) Fh[q] = 0.5 * (FL[q] + FR[q]) - 0.5 * s * (UR[q] - UL[q]);
}

// U^(i) = U^n - dt sum_j c_j Phi(U^(j)) on fluid cells (eqs. RKEuler, RKEuler_2).
// One tile of cells per 4-wavefront block.  Only the newest state's flux
// divergence is formed: its tile with the 2-cell periodic halo is staged in
// LDS, every face flux of the tile is computed once ((ET + 1) x ET faces per
// direction, one thread per face, so the divide / square-root chains of many
// faces interleave), each cell takes the difference of its two faces per
// direction and stores it for the later stages of the step; the divergences
// of earlier states are read back (each state's is formed once per step).
// Tiles of ET x ET cells: 8 x 8, or 16 x 16 on grids of at least 1024 such
// tiles (fewer halo cells and idle face threads per cell; measured 23% faster
// at 1024^2 cells, slower at 256^2 where 16 x 16 tiles leave CUs idle).
constexpr int EH = 2, ENT = 256, ENJ = 3;
constexpr long kEulerBigTiles = 1024;

template <int ET>
__global__ __launch_bounds__(ENT) void euler_stage_kernel(EulerArgs a) {
    constexpr int EW = ET + 2 * EH;
    constexpr int EFACES = ET * (ET + 1);  // faces per direction
    static_assert(ET * ET <= ENT, "one thread per cell of the tile");
    __shared__ double u[1][4][EW][EW];
    __shared__ double fx[1][4][ET][ET + 1];
    __shared__ double fy[1][4][ET + 1][ET];
    const int tid = (int)threadIdx.x;
    const int i0 = (int)blockIdx.x * ET, j0 = (int)blockIdx.y * ET;
    const int nx = a.nx, ny = a.ny, nj = a.nj;
    const int jn = a.jnew;  // the one state whose divergence is formed here (-1: none)
    const size_t nc = (size_t)a.nc;
    // cell of threads 0..63
    const int tx = tid % ET, ty = tid / ET;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = tid < ET * ET && i < nx && j < ny;
    const size_t cell = own ? (size_t)j * nx + i : 0;
    const bool fluid = own && !a.mask[cell];
    if (!__syncthreads_or(fluid)) return;  // whole tile kinetic (or outside)
    const int nnew = jn >= 0 ? 1 : 0;
    for (int t = tid; t < nnew * EW * EW; t += ENT) {
        const int jj = 0, r = t;
        const int li = r % EW, lj = r / EW;
        const int gi = wrapc(i0 + li - EH, nx), gj = wrapc(j0 + lj - EH, ny);
        const size_t c = (size_t)gj * nx + gi;
        const double *U = a.Uj[jn];
#pragma unroll
        for (int q = 0; q < 4; ++q) u[jj][q][lj][li] = U[q * nc + c];
    }
    __syncthreads();
    for (int t = tid; t < nnew * 2 * EFACES; t += ENT) {
        const int jj = 0, r = t;
        const int d = r / EFACES, k = r % EFACES;
        double st[4][4], F[4];
        if (d == 0) {
            // x-face f (0..8) of row rr lies between local cells f-1 and f
            const int rr = k / (ET + 1), f = k % (ET + 1);
            const int y = rr + EH, x = f + EH;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                st[q][0] = u[jj][q][y][x - 2]; st[q][1] = u[jj][q][y][x - 1];
                st[q][2] = u[jj][q][y][x]; st[q][3] = u[jj][q][y][x + 1];
            }
            euler_face_vals(st, 0, a.recon, F);
#pragma unroll
            for (int q = 0; q < 4; ++q) fx[jj][q][rr][f] = F[q];
        } else {
            const int f = k / ET, cidx = k % ET;
            const int y = f + EH, x = cidx + EH;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                st[q][0] = u[jj][q][y - 2][x]; st[q][1] = u[jj][q][y - 1][x];
                st[q][2] = u[jj][q][y][x]; st[q][3] = u[jj][q][y + 1][x];
            }
            euler_face_vals(st, 1, a.recon, F);
#pragma unroll
            for (int q = 0; q < 4; ++q) fy[jj][q][f][cidx] = F[q];
        }
    }
    __syncthreads();
    if (fluid) {
        const double idx = 1.0 / a.dx, idy = 1.0 / a.dy;
        double s[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] = a.Un[q * nc + cell];
        for (int jj = 0; jj < nj; ++jj) {
            const double c = a.dt * a.cj[jj];
            double D[4];
            if (jj == jn) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    D[q] = (fx[0][q][ty][tx + 1] - fx[0][q][ty][tx]) * idx +
                           (fy[0][q][ty + 1][tx] - fy[0][q][ty][tx]) * idy;
                if (a.Dout) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) a.Dout[q * nc + cell] = D[q];
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) D[q] = a.Dj[jj][q * nc + cell];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] -= c * D[q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) a.Uout[q * nc + cell] = s[q];
    }
}

// Every floating-point expression from here on is evaluated as written: no
// fused multiply-add contraction (the indicator's results must be the
// correctly rounded IEEE operations of its documented order).
#pragma clang fp contract(off)

// ------------------------------------------------------- conversions

// Primitive variables, every operation a correctly rounded IEEE double op in
// a fixed order (part of the bit-exact indicator contract; this file is
// compiled without contraction, and the expressions are written with plain
// operators in it so that the setting applies to them).
__device__ inline void prim_of(double U0, double U1, double U2, double U3, double *rho, double *ux,
                               double *uy, double *T) {
    *rho = U0;
    *ux = U1 / U0;
    *uy = U2 / U0;
    const double k = (0.5 * U0) * ((*ux) * (*ux) + (*uy) * (*uy));
    *T = (U3 - k) / U0;
}

__global__ void prim_kernel(const double *U, double *prim, int nc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const size_t n = (size_t)nc;
    double r, ux, uy, T;
    prim_of(U[c], U[n + c], U[2 * n + c], U[3 * n + c], &r, &ux, &uy, &T);
    prim[c] = r; prim[n + c] = ux; prim[2 * n + c] = uy; prim[3 * n + c] = T;
}

__global__ void conserved_kernel(const double *rho, const double *ux, const double *uy,
                                 const double *T, const double *eps, double *U, double *eps_out,
                                 int nc, int *bad) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const size_t n = (size_t)nc;
    double r = rho[c], a = ux[c], b = uy[c], t = T[c], e = eps[c];
    if (!(r > 0.0) || !(t > 0.0) || !(e > 0.0) || !isfinite(r) || !isfinite(a) || !isfinite(b) ||
        !isfinite(t) || !isfinite(e))
        atomicOr(bad, 1);
    U[c] = r;
    U[n + c] = r * a;
    U[2 * n + c] = r * b;
    U[3 * n + c] = 0.5 * r * (a * a + b * b) + r * t;
    eps_out[c] = e;
}

// ------------------------------------------------------------- indicator

// Regime indicator of Sec. 3.1.2 at one cell.  The operation order matches the
// documented contract (plain operators in this no-contraction file, correctly
// rounded + - * / only: the
// criterion lambda > eta is decided through the square-root-free equivalent
// eta - |m| < 0 or q > (eta - |m|)^2, and (ck eps/(tau sqrt T))^2 is formed as
// (ck eps)^2 / (tau^2 T)).
__device__ inline uint8_t indicator_cell(const IndicatorArgs &a, int cell, double *lam_out) {
    const size_t n = (size_t)a.nc;
    const int nx = a.nx, ny = a.ny;
    const int i = cell % nx, j = cell / nx;
    const size_t ce = (size_t)j * nx + wrapc(i + 1, nx), cw = (size_t)j * nx + wrapc(i - 1, nx);
    const size_t cn = (size_t)wrapc(j + 1, ny) * nx + i, cs = (size_t)wrapc(j - 1, ny) * nx + i;
    // primitives of the 5-point stencil: read, or formed from U with prim_of
    double pux[5], puy[5], pT[5];  // order: centre, e, w, n, s
    const size_t st[5] = {(size_t)cell, ce, cw, cn, cs};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if (a.U) {
            double r;
            prim_of(a.U[st[q]], a.U[n + st[q]], a.U[2 * n + st[q]], a.U[3 * n + st[q]], &r, &pux[q], &puy[q], &pT[q]);
        } else {
            pux[q] = a.prim[n + st[q]];
            puy[q] = a.prim[2 * n + st[q]];
            pT[q] = a.prim[3 * n + st[q]];
        }
    }
    const double twodx = a.twodx, twody = a.twody;
    const double uxx = (pux[1] - pux[2]) / twodx;
    const double uxy = (pux[3] - pux[4]) / twody;
    const double uyx = (puy[1] - puy[2]) / twodx;
    const double uyy = (puy[3] - puy[4]) / twody;
    const double Tx = (pT[1] - pT[2]) / twodx;
    const double Ty = (pT[3] - pT[4]) / twody;
    const double div = uxx + uyy;
    const double Dxx = (uxx + uxx) - a.cD * div;
    const double Dxy = uxy + uyx;
    const double Dyy = (uyy + uyy) - a.cD * div;
    const double e = a.eps[cell];
    const double cv = e / (a.tau * a.omb);
    const double ke = a.ck * e;
    const double kt2 = a.cS * ((ke * ke) / ((a.tau * a.tau) * pT[0]));
    const double a11 = -(cv * Dxx) - kt2 * (Tx * Tx);
    const double a12 = -(cv * Dxy) - kt2 * (Tx * Ty);
    const double a22 = -(cv * Dyy) - kt2 * (Ty * Ty);
    const double m = (a11 + a22) / 2.0;
    const double h = (a11 - a22) / 2.0;
    const double q = h * h + a12 * a12;
    if (lam_out) *lam_out = fabs(m) + sqrt(q);  // report only
    // |m| + sqrt(q) > eta  <=>  eta - |m| < 0  or  q > (eta - |m|)^2: no square root decides
    const double dd = a.eta - fabs(m);
    const bool critS = (dd < 0.0) || (q > dd * dd);
    const bool critL = a.l1[cell] > a.delta;
    return (uint8_t)(critS || (a.mask_old[cell] && critL));
}

__global__ void indicator_kernel(IndicatorArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.nc) return;
    double lam;
    uint8_t m = indicator_cell(a, c, &lam);
    a.mask_new[c] = m;
    if (a.lambda) a.lambda[c] = lam;
}

// ------------------------------------------------- classify + compaction

// class bits: 1 kinetic, 2 buffer (fluid cell inside a kinetic stencil),
// 4 newly kinetic (needs f = Mhat(U)).

// Position -> cell in the processing order: 8x8 cell tiles, row-major inside
// a tile, tiles row-major; -1 for positions of a padded edge tile.
__device__ inline int pos_to_cell(int pos, int nx, int ny) {
    const int ntx = (nx + 7) / 8;
    const int t = pos >> 6, w = pos & 63;
    const int i = (t % ntx) * 8 + (w & 7), j = (t / ntx) * 8 + (w >> 3);
    return (i < nx && j < ny) ? j * nx + i : -1;
}

constexpr int kScanBlock = 1024;  // positions per block, one per thread

__device__ inline uint8_t class_of(const uint8_t *mask, const uint8_t *mask_old, int c, int nx, int ny, int radius) {
    const int i = c % nx, j = c / nx;
    uint8_t out = 0;
    if (mask[c]) {
        out = 1;
        if (mask_old && !mask_old[c]) out |= 4;
    } else {
        bool near = false;
        for (int d = 1; d <= radius; ++d) {
            near = near || mask[(size_t)j * nx + wrapc(i - d, nx)] || mask[(size_t)j * nx + wrapc(i + d, nx)] ||
                   mask[(size_t)wrapc(j - d, ny) * nx + i] || mask[(size_t)wrapc(j + d, ny) * nx + i];
        }
        if (near) out = 2;
    }
    return out;
}

// Classification of every cell (written to cls) and the per-block counts of
// the three classes in processing order.
__global__ __launch_bounds__(kScanBlock) void classify_count_kernel(const uint8_t *mask, const uint8_t *mask_old,
                                                                    uint8_t *cls, int radius, int nx, int ny,
                                                                    int npos, int *blockcounts, int nblocks) {
    const int t = threadIdx.x;
    const int pos = blockIdx.x * kScanBlock + t;
    uint8_t k = 0;
    if (pos < npos) {
        const int cell = pos_to_cell(pos, nx, ny);
        if (cell >= 0) {
            k = class_of(mask, mask_old, cell, nx, ny, radius);
            cls[cell] = k;
        }
    }
    const int n1 = __syncthreads_count((k & 1) != 0);
    const int n2 = __syncthreads_count((k & 2) != 0);
    const int n4 = __syncthreads_count((k & 4) != 0);
    if (t == 0) {
        blockcounts[blockIdx.x] = n1;
        blockcounts[nblocks + blockIdx.x] = n2;
        blockcounts[2 * nblocks + blockIdx.x] = n4;
    }
}

// Scatter of the three lists in processing order.  Each block first sums
// the counts of the blocks before it (a fixed-order reduction, so the lists
// are deterministic); the last block writes the totals to counts[0..2] and
// adds the kinetic count to *total (when given).
__global__ __launch_bounds__(kScanBlock) void scan_scatter_kernel(const uint8_t *cls, int nx, int ny, int npos,
                                                                  const int *blockcounts, int nblocks, int *kin,
                                                                  int *buf, int *newk, int *counts, long long *total) {
    __shared__ int sc[3][kScanBlock];
    __shared__ int boff[3];
    const int t = threadIdx.x;
    {
        int part[3] = {0, 0, 0};
        for (int b = t; b < (int)blockIdx.x; b += kScanBlock)
#pragma unroll
            for (int q = 0; q < 3; ++q) part[q] += blockcounts[q * nblocks + b];
#pragma unroll
        for (int q = 0; q < 3; ++q) sc[q][t] = part[q];
        __syncthreads();
        for (int s2 = kScanBlock / 2; s2 > 0; s2 >>= 1) {
            if (t < s2)
#pragma unroll
                for (int q = 0; q < 3; ++q) sc[q][t] += sc[q][t + s2];
            __syncthreads();
        }
        if (t < 3) boff[t] = sc[t][0];
        __syncthreads();
    }
    const int pos = blockIdx.x * kScanBlock + t;
    const int cell = pos < npos ? pos_to_cell(pos, nx, ny) : -1;
    const uint8_t k = cell >= 0 ? cls[cell] : 0;
    int loc[3] = {(k & 1) != 0, (k & 2) != 0, (k & 4) != 0};
    // inclusive scan of the block's flags (Hillis-Steele in LDS)
#pragma unroll
    for (int q = 0; q < 3; ++q) sc[q][t] = loc[q];
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int add[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) add[q] = t >= off ? sc[q][t - off] : 0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) sc[q][t] += add[q];
        __syncthreads();
    }
    if (k & 1) kin[boff[0] + sc[0][t] - 1] = cell;
    if (k & 2) buf[boff[1] + sc[1][t] - 1] = cell;
    if (k & 4) newk[boff[2] + sc[2][t] - 1] = cell;
    if ((int)blockIdx.x == nblocks - 1 && t == kScanBlock - 1) {
        for (int q = 0; q < 3; ++q) counts[q] = boff[q] + sc[q][t];
        if (total) *total += boff[0] + sc[0][t];
    }
}

__global__ void get_prim_kernel(const double *U, double *rho, double *ux, double *uy, double *T, int nc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const size_t n = (size_t)nc;
    double r, a, b, t;
    prim_of(U[c], U[n + c], U[2 * n + c], U[3 * n + c], &r, &a, &b, &t);
    if (rho) rho[c] = r;
    if (ux) ux[c] = a;
    if (uy) uy[c] = b;
    if (T) T[c] = t;
}

__global__ void zero_fluid_l1_kernel(const uint8_t *mask, double *l1, int nc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc && !mask[c]) l1[c] = 0.0;
}

__global__ void accumulate_count_kernel(const int *counts, long long *total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *total += counts[0];
}

// ------------------------------------------------------- host launchers

static inline unsigned cells_grid(int n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

// ------------------------------------------------- learned indicator glue

__device__ inline void count_add(long long *counters, int q, bool pred) {
    const int n = __syncthreads_count(pred);
    if (threadIdx.x == 0 && n) atomicAdd((unsigned long long *)&counters[q], (unsigned long long)n);
}

// Mask of a check step: plain | (logit > threshold), or the plain mask
// dilated by r cells (r > 0: this pass takes the maximum along x into tmp).
__global__ void learned_combine_kernel(const uint8_t *plain, const float *logits, float threshold, int r,
                                       const uint8_t *in_use, uint8_t *out, uint8_t *tmp, int nx, int ny,
                                       long long *counters) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int nc = nx * ny;
    const bool live = c < nc;
    const bool p = live && plain[c];
    if (live) {
        if (r > 0) {
            const int i = c % nx, j = c / nx;
            uint8_t m = 0;
            for (int d = -r; d <= r; ++d) m |= plain[(size_t)j * nx + wrapc(i + d, nx)];
            tmp[c] = m;
        } else {
            out[c] = (uint8_t)(p || (logits && logits[c] > threshold));
        }
    }
    if (counters) {
        const bool u = live && in_use[c];
        count_add(counters, 1, p && !u);
        count_add(counters, 2, u && !p);
        count_add(counters, 3, p);
        if (c == 0) atomicAdd((unsigned long long *)&counters[0], 1ull);
    }
}

// Second pass of the dilation: maximum along y.
__global__ void dilate_y_kernel(const uint8_t *tmp, uint8_t *out, int nx, int ny, int r) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nx * ny) return;
    const int i = c % nx, j = c / nx;
    uint8_t m = 0;
    for (int d = -r; d <= r; ++d) m |= tmp[(size_t)wrapc(j + d, ny) * nx + i];
    out[c] = m;
}


hipError_t launch_euler(const EulerArgs &a, hipStream_t st) {
    if (a.nj < 0 || a.nj > ENJ || a.jnew >= a.nj) return hipErrorInvalidValue;
    for (int j = 0; j < a.nj; ++j)
        if (j != a.jnew && !a.Dj[j]) return hipErrorInvalidValue;
    const long big = (long)((a.nx + 15) / 16) * ((a.ny + 15) / 16);
    if (big >= kEulerBigTiles) {
        const dim3 grid((unsigned)((a.nx + 15) / 16), (unsigned)((a.ny + 15) / 16));
        hipLaunchKernelGGL(euler_stage_kernel<16>, grid, dim3(ENT), 0, st, a);
    } else {
        const dim3 grid((unsigned)((a.nx + 7) / 8), (unsigned)((a.ny + 7) / 8));
        hipLaunchKernelGGL(euler_stage_kernel<8>, grid, dim3(ENT), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_prim(const double *U, double *prim, int nc, hipStream_t st) {
    hipLaunchKernelGGL(prim_kernel, dim3(cells_grid(nc)), dim3(256), 0, st, U, prim, nc);
    return hipGetLastError();
}

hipError_t launch_conserved(const double *rho, const double *ux, const double *uy, const double *T,
                            const double *eps, double *U, double *eps_out, int nc, int *bad,
                            hipStream_t st) {
    hipLaunchKernelGGL(conserved_kernel, dim3(cells_grid(nc)), dim3(256), 0, st, rho, ux, uy, T, eps, U,
                       eps_out, nc, bad);
    return hipGetLastError();
}

hipError_t launch_indicator(const IndicatorArgs &a, hipStream_t st) {
    hipLaunchKernelGGL(indicator_kernel, dim3(cells_grid(a.nc)), dim3(256), 0, st, a);
    return hipGetLastError();
}

int scan_positions(int nx, int ny) { return ((nx + 7) / 8) * ((ny + 7) / 8) * 64; }
int scan_nblocks(int nx, int ny) { return (scan_positions(nx, ny) + kScanBlock - 1) / kScanBlock; }

hipError_t launch_compact(const uint8_t *mask, const uint8_t *mask_old, uint8_t *cls, int radius, int nx, int ny,
                          int *blockcounts, int *counts, int *kin, int *buf, int *newk, long long *total,
                          hipStream_t st) {
    const int npos = scan_positions(nx, ny), nb = scan_nblocks(nx, ny);
    hipLaunchKernelGGL(classify_count_kernel, dim3(nb), dim3(kScanBlock), 0, st, mask, mask_old, cls, radius, nx, ny,
                       npos, blockcounts, nb);
    hipLaunchKernelGGL(scan_scatter_kernel, dim3(nb), dim3(kScanBlock), 0, st, cls, nx, ny, npos, blockcounts, nb, kin,
                       buf, newk, counts, total);
    return hipGetLastError();
}

hipError_t launch_get_prim(const double *U, double *rho, double *ux, double *uy, double *T, int nc,
                           hipStream_t st) {
    hipLaunchKernelGGL(get_prim_kernel, dim3(cells_grid(nc)), dim3(256), 0, st, U, rho, ux, uy, T, nc);
    return hipGetLastError();
}

hipError_t launch_accumulate_count(const int *counts, long long *total, hipStream_t st) {
    hipLaunchKernelGGL(accumulate_count_kernel, dim3(1), dim3(64), 0, st, counts, total);
    return hipGetLastError();
}

hipError_t launch_zero_fluid_l1(const uint8_t *mask, double *l1, int nc, hipStream_t st) {
    hipLaunchKernelGGL(zero_fluid_l1_kernel, dim3(cells_grid(nc)), dim3(256), 0, st, mask, l1, nc);
    return hipGetLastError();
}

hipError_t launch_learned_combine(const uint8_t *plain, const float *logits, float threshold, int dilation,
                                  const uint8_t *in_use, uint8_t *out, uint8_t *tmp, int nx, int ny,
                                  long long *counters, hipStream_t st) {
    const int nc = nx * ny;
    hipLaunchKernelGGL(learned_combine_kernel, dim3(cells_grid(nc)), dim3(256), 0, st, plain, logits, threshold,
                       dilation, in_use, out, tmp, nx, ny, counters);
    if (dilation > 0)
        hipLaunchKernelGGL(dilate_y_kernel, dim3(cells_grid(nc)), dim3(256), 0, st, tmp, out, nx, ny, dilation);
    return hipGetLastError();
}


}  // namespace esbgk
