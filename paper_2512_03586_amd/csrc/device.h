// device.h -- device-side building blocks of the MI355X kinetic IMEX engine.
//
// Work decomposition used by every phase-space kernel: one 64-lane wavefront
// owns one cell's whole velocity block (nv*nv values, velocity-contiguous in
// HBM).  Lane l owns "chunks" of 4 consecutive nodes k0 = 4*(l + 64*m),
// m = 0..C-1, so a wavefront load instruction reads 64 x 16 B (FP32) of
// contiguous memory.  nv is a multiple of 4, hence the 4 nodes of a chunk
// share the same y-velocity.  Velocity reductions (moments, Gram sums) are
// per-lane partial sums over the lane's chunks followed by a butterfly across
// the wavefront; the butterfly only relies on commutativity of IEEE addition,
// so every lane ends with the bit-identical total.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace esbgk {

constexpr double kPi = 3.14159265358979323846;
constexpr double kLog2e = 1.44269504088896340736;

// ---------------------------------------------------------------- storage

struct bf16_t { uint16_t bits; };

template <class S> struct Storage;

template <> struct Storage<double> {
    using T = double;  // arithmetic type
    __device__ static inline void load4(const double *p, size_t idx, double v[4]) {
        const double2 *q = reinterpret_cast<const double2 *>(p + idx);
        double2 a = q[0], b = q[1];
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
    __device__ static inline void store4(double *p, size_t idx, const double v[4]) {
        double2 *q = reinterpret_cast<double2 *>(p + idx);
        q[0] = make_double2(v[0], v[1]);
        q[1] = make_double2(v[2], v[3]);
    }
};

template <> struct Storage<float> {
    using T = float;
    __device__ static inline void load4(const float *p, size_t idx, float v[4]) {
        float4 a = *reinterpret_cast<const float4 *>(p + idx);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    }
    __device__ static inline void store4(float *p, size_t idx, const float v[4]) {
        *reinterpret_cast<float4 *>(p + idx) = make_float4(v[0], v[1], v[2], v[3]);
    }
};

__device__ inline float bf16_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

// round to nearest even (finite inputs)
__device__ inline uint32_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

template <> struct Storage<bf16_t> {
    using T = float;
    __device__ static inline void load4(const bf16_t *p, size_t idx, float v[4]) {
        uint2 a = *reinterpret_cast<const uint2 *>(p + idx);
        v[0] = bf16_to_f32(a.x & 0xFFFFu); v[1] = bf16_to_f32(a.x >> 16);
        v[2] = bf16_to_f32(a.y & 0xFFFFu); v[3] = bf16_to_f32(a.y >> 16);
    }
    __device__ static inline void store4(bf16_t *p, size_t idx, const float v[4]) {
        uint2 a;
        a.x = f32_to_bf16(v[0]) | (f32_to_bf16(v[1]) << 16);
        a.y = f32_to_bf16(v[2]) | (f32_to_bf16(v[3]) << 16);
        *reinterpret_cast<uint2 *>(p + idx) = a;
    }
};

// --------------------------------------------------------- scalar helpers

__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline double fast_exp2(double x) { return exp2(x); }

// minmod(a, b) = median(a, b, 0)
__device__ inline float minmod(float a, float b) { return __builtin_amdgcn_fmed3f(a, b, 0.0f); }
__device__ inline double minmod(double a, double b) { return fmax(fmin(a, b), fmin(fmax(a, b), 0.0)); }

// --------------------------------------------------------- wave reductions

template <class T> __device__ inline T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Compensated (hi, lo) accumulator in the arithmetic type: TwoSum keeps the
// exact rounding error of every addition in lo.
template <class T> struct Comp {
    T hi, lo;
    __device__ inline Comp() : hi(0), lo(0) {}
    __device__ inline void add(T x) {
        T s = hi + x;
        T bb = s - hi;
        T e = (hi - (s - bb)) + (x - bb);
        hi = s;
        lo += e;
    }
    __device__ inline void merge(T ohi, T olo) {
        T s = hi + ohi;
        T bb = s - hi;
        T e = (hi - (s - bb)) + (ohi - bb);
        hi = s;
        lo = (lo + olo) + e;
    }
    __device__ inline double value() const { return (double)hi + (double)lo; }
};

template <class T> __device__ inline double wave_sum_comp(Comp<T> c) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T ohi = __shfl_xor(c.hi, off, 64);
        T olo = __shfl_xor(c.lo, off, 64);
        // merge symmetrically: TwoSum's error term is exact, so (a,b) and (b,a)
        // give identical results in both lanes of a pair
        c.merge(ohi, olo);
    }
    return c.value();
}

// -------------------------------------------------------- kernel geometry

struct Geom {
    int nx, ny, nv, nv2;
    double dx, dy, dv, vmax, w;  // w = dv^2 quadrature weight
    double beta, tau, dt;
    int recon, correction;
};

// Chunk m of lane l: first node index, and whether it exists.
__device__ inline int chunk_node(int lane, int m) { return 4 * (lane + 64 * m); }

// ------------------------------------------ per-cell Gaussian parameters
//
// A sampled Gaussian with the conservation correction is stored per cell as
// 16 doubles so that later kernels can re-evaluate it at any node without
// touching the velocity block:
//   Ghat(v) = exp2(l2p + qxx xi_x^2 + qxy xi_x xi_y + qyy xi_y^2) * (c . psi),
//   xi = v - u, psi = (1, a, b, a^2, a b, b^2), (a, b) = xi / sqrt(T).
enum GP { GP_UX = 0, GP_UY, GP_QXX, GP_QXY, GP_QYY, GP_L2P, GP_IST, GP_C0, GP_C1, GP_C2,
          GP_C3, GP_C4, GP_C5, GP_RHO, GP_T, GP_PAD, GP_N };

// Fill the exponent part of the parameters of the Gaussian with density rho,
// mean u and covariance tensor Tt (Sec. 2: rho / sqrt(det(2 pi Tt)) *
// exp(-xi^T Tt^{-1} xi / 2)), all in FP64.  Returns false if Tt is not SPD.
__device__ inline bool gauss_params(double rho, double ux, double uy, double T, double txx,
                                    double txy, double tyy, double *gp) {
    double det = txx * tyy - txy * txy;
    bool ok = det > 0.0 && txx > 0.0 && rho > 0.0 && T > 0.0;
    double idet = 1.0 / det;
    double ixx = tyy * idet, ixy = -txy * idet, iyy = txx * idet;
    gp[GP_UX] = ux;
    gp[GP_UY] = uy;
    gp[GP_QXX] = -0.5 * kLog2e * ixx;
    gp[GP_QXY] = -kLog2e * ixy;
    gp[GP_QYY] = -0.5 * kLog2e * iyy;
    gp[GP_L2P] = log2(rho / (2.0 * kPi * sqrt(det)));
    gp[GP_IST] = 1.0 / sqrt(T);
    gp[GP_C0] = 1.0;
    gp[GP_C1] = gp[GP_C2] = gp[GP_C3] = gp[GP_C4] = gp[GP_C5] = 0.0;
    gp[GP_RHO] = rho;
    gp[GP_T] = T;
    gp[GP_PAD] = 0.0;
    return ok;
}

// Unknowns of the conservation correction from the 15 discrete moments
// S_pq = w sum Gtilde a^p b^q (p + q <= 4) of the sampled Gaussian: the Gram
// matrix A_mn = w sum Gtilde psi_m psi_n and the target moments
// t = (rho, 0, 0, rho txx/T, rho txy/T, rho tyy/T).  Writes c into gp[GP_C0..].
// Solved in deviation form A dc = t - A e0 (c = e0 + dc) by Cholesky in FP64.
__device__ inline bool solve_correction(const double S[15], double rho, double T, double txx,
                                        double txy, double tyy, double *gp) {
    // monomial index of a^p b^q in S: order (00,10,01,20,11,02,30,21,12,03,40,31,22,13,04)
    const int pp[6] = {0, 1, 0, 2, 1, 0}, qq[6] = {0, 0, 1, 0, 1, 2};
    auto mon = [&](int p, int q) -> double {
        int d = p + q;
        int base = d * (d + 1) / 2;  // 0,1,3,6,10
        return S[base + q];
    };
    double A[6][6];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int n = 0; n < 6; ++n) A[m][n] = mon(pp[m] + pp[n], qq[m] + qq[n]);
    double r[6];
    double iT = 1.0 / T;
    r[0] = rho - A[0][0];
    r[1] = -A[1][0];
    r[2] = -A[2][0];
    r[3] = rho * txx * iT - A[3][0];
    r[4] = rho * txy * iT - A[4][0];
    r[5] = rho * tyy * iT - A[5][0];
    // Cholesky A = L L^T (in place, lower triangle)
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
        ok = ok && d > 0.0;
        double ljj = sqrt(d);
        A[j][j] = ljj;
        double il = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k];
            A[i][j] = s * il;
        }
    }
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = r[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= A[i][k] * y[k];
        y[i] = s / A[i][i];
    }
    double x[6];
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= A[k][i] * x[k];
        x[i] = s / A[i][i];
    }
    if (ok) {
        gp[GP_C0] = 1.0 + x[0];
        gp[GP_C1] = x[1];
        gp[GP_C2] = x[2];
        gp[GP_C3] = x[3];
        gp[GP_C4] = x[4];
        gp[GP_C5] = x[5];
    }
    return ok;
}

// Per-lane copy of a cell's Gaussian parameters in the arithmetic type.
template <class T> struct GaussEval {
    T ux, uy, qxx, qxy, qyy, l2p, ist, c0, c1, c2, c3, c4, c5;
    __device__ inline void load(const double *gp) {
        ux = (T)gp[GP_UX]; uy = (T)gp[GP_UY];
        qxx = (T)gp[GP_QXX]; qxy = (T)gp[GP_QXY]; qyy = (T)gp[GP_QYY];
        l2p = (T)gp[GP_L2P]; ist = (T)gp[GP_IST];
        c0 = (T)gp[GP_C0]; c1 = (T)gp[GP_C1]; c2 = (T)gp[GP_C2];
        c3 = (T)gp[GP_C3]; c4 = (T)gp[GP_C4]; c5 = (T)gp[GP_C5];
    }
    // sampled Gaussian (no correction)
    __device__ inline T tilde(T vx, T vy) const {
        T ex = vx - ux, ey = vy - uy;
        return fast_exp2(l2p + (qxx * ex + qxy * ey) * ex + qyy * ey * ey);
    }
    __device__ inline T poly(T vx, T vy) const {
        T a = (vx - ux) * ist, b = (vy - uy) * ist;
        return c0 + (c1 + c3 * a + c4 * b) * a + (c2 + c5 * b) * b;
    }
    __device__ inline T hat(T vx, T vy) const { return tilde(vx, vy) * poly(vx, vy); }
};

// error flag bits
enum { ERR_RHO = 1, ERR_T = 2, ERR_SPD = 4, ERR_NAN = 8 };

}  // namespace esbgk
