// device.h -- device-side building blocks of the MI355X kinetic IMEX engine.
//
// Work decomposition of every phase-space kernel: a group of L lanes
// (L = 16, 32 or 64; a 16-lane group is one DPP row) owns one cell's whole
// velocity block (nv*nv values, velocity-contiguous in HBM), so a 64-lane
// wavefront works on 64/L cells at once.  Lane s of a group owns the chunks of
// 4 consecutive nodes k0 = 4*(s + L*m), m = 0..C-1; nv is a multiple of 4, so
// the 4 nodes of a chunk share one y-velocity.  A velocity reduction is a
// per-lane partial sum followed by a butterfly inside the group made of DPP
// lane permutations (plus one ds_swizzle / readlane step for 32- and 64-lane
// groups); every butterfly step adds a pair of lanes symmetrically, and IEEE
// addition is commutative, so every lane of a group ends with the
// bit-identical total.  The per-cell FP64 algebra after a reduction therefore
// runs once per wavefront for all of its cells.
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
    template <class I> __device__ static inline void load4(const double *p, I idx, double v[4]) {
        const double2 *q = reinterpret_cast<const double2 *>(p + idx);
        double2 a = q[0], b = q[1];
        v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
    template <class I> __device__ static inline void store4(double *p, I idx, const double v[4]) {
        double2 *q = reinterpret_cast<double2 *>(p + idx);
        q[0] = make_double2(v[0], v[1]);
        q[1] = make_double2(v[2], v[3]);
    }
};

template <> struct Storage<float> {
    using T = float;
    template <class I> __device__ static inline void load4(const float *p, I idx, float v[4]) {
        float4 a = *reinterpret_cast<const float4 *>(p + idx);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    }
    template <class I> __device__ static inline void store4(float *p, I idx, const float v[4]) {
        *reinterpret_cast<float4 *>(p + idx) = make_float4(v[0], v[1], v[2], v[3]);
    }
};

// round to nearest even (finite inputs)
__device__ inline uint32_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

template <> struct Storage<bf16_t> {
    using T = float;
    template <class I> __device__ static inline void load4(const bf16_t *p, I idx, float v[4]) {
        uint2 a = *reinterpret_cast<const uint2 *>(p + idx);
        v[0] = __uint_as_float(a.x << 16); v[1] = __uint_as_float(a.x & 0xFFFF0000u);
        v[2] = __uint_as_float(a.y << 16); v[3] = __uint_as_float(a.y & 0xFFFF0000u);
    }
    template <class I> __device__ static inline void store4(bf16_t *p, I idx, const float v[4]) {
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

// ------------------------------------------------------ group reductions

template <int CTRL> __device__ inline uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
__device__ inline uint32_t swz_xor16(uint32_t v) {
    // ds_swizzle bit-mask mode inside 32-lane halves: and 0x1F, or 0, xor 0x10
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x401F);
}

// Value of the partner lane at butterfly step STEP:
// 0: lane^1, 1: lane^2 (quad permutes), 2: half-row mirror, 3: row mirror,
// 4: lane^16 (32-lane halves).
template <int STEP> __device__ inline uint32_t partner32(uint32_t v) {
    if constexpr (STEP == 0) return dpp32<0xB1>(v);   // quad_perm [1,0,3,2]
    else if constexpr (STEP == 1) return dpp32<0x4E>(v);  // quad_perm [2,3,0,1]
    else if constexpr (STEP == 2) return dpp32<0x141>(v); // row_half_mirror
    else if constexpr (STEP == 3) return dpp32<0x140>(v); // row_mirror
    else return swz_xor16(v);
}

template <int STEP> __device__ inline float partner(float v) {
    return __uint_as_float(partner32<STEP>(__float_as_uint(v)));
}
template <int STEP> __device__ inline double partner(double v) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t lo = partner32<STEP>((uint32_t)u), hi = partner32<STEP>((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ inline float readlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline double readlane(double v, int l) {
    uint64_t u = (uint64_t)__double_as_longlong(v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the L lanes of a group; every lane of the group gets the same value.
template <int L, class T> __device__ inline T group_sum(T v) {
    v += partner<0>(v);
    v += partner<1>(v);
    v += partner<2>(v);
    v += partner<3>(v);
    if constexpr (L >= 32) v += partner<4>(v);
    if constexpr (L == 64) v = readlane(v, 0) + readlane(v, 32);
    return v;
}

// Compensated (hi, lo) pair: TwoSum keeps the exact rounding error of every
// addition in lo.  merge() is symmetric in its operands (the TwoSum error term
// is exact), so a butterfly of merges leaves identical pairs in all lanes.
template <class T> struct Comp {
    T hi = 0, lo = 0;
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

#ifndef ESBGK_COMP_BUTTERFLY
#define ESBGK_COMP_BUTTERFLY 0
#endif

// Group total of compensated lane partials.  Default: each lane's (hi + lo) is
// formed in FP64 and the butterfly adds in FP64 (about 64 * 2^-53 relative
// error, far below the FP32 partials' own), a third of the instructions of a
// butterfly of TwoSum merges.
template <int L, class T> __device__ inline double group_sum_comp(Comp<T> c) {
    if constexpr (ESBGK_COMP_BUTTERFLY == 0) {
        return group_sum<L>((double)c.hi + (double)c.lo);
    } else {
        c.merge(partner<0>(c.hi), partner<0>(c.lo));
        c.merge(partner<1>(c.hi), partner<1>(c.lo));
        c.merge(partner<2>(c.hi), partner<2>(c.lo));
        c.merge(partner<3>(c.hi), partner<3>(c.lo));
        if constexpr (L >= 32) c.merge(partner<4>(c.hi), partner<4>(c.lo));
        if constexpr (L == 64) {
            T h0 = readlane(c.hi, 0), l0 = readlane(c.lo, 0);
            T h1 = readlane(c.hi, 32), l1 = readlane(c.lo, 32);
            Comp<T> r;
            r.hi = h0; r.lo = l0;
            r.merge(h1, l1);
            return r.value();
        }
        return c.value();
    }
}

// Wave-wide totals of six doubles, each lane's six values in, every lane gets
// all six totals.  A transposed butterfly: the 32-lane halves exchange whole
// values (v_permlane32_swap: lanes 32-63 of one operand with lanes 0-31 of the
// other), so after one add the low half holds x[q] and the high half x[q+3];
// the odd/even 16-lane rows do the same (v_permlane16_swap), then four DPP
// steps finish inside each row and six readlanes collect the totals.  Each
// total is one fixed tree over the 64 lanes.
__device__ inline void swap_halves(double &a, double &b, bool rows16) {
    const uint64_t ua = (uint64_t)__double_as_longlong(a), ub = (uint64_t)__double_as_longlong(b);
    uint32_t alo = (uint32_t)ua, ahi = (uint32_t)(ua >> 32), blo = (uint32_t)ub, bhi = (uint32_t)(ub >> 32);
    if (rows16) {
        auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
        auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
        alo = lo[0]; blo = lo[1]; ahi = hi[0]; bhi = hi[1];
    } else {
        auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
        auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
        alo = lo[0]; blo = lo[1]; ahi = hi[0]; bhi = hi[1];
    }
    a = __longlong_as_double((long long)(((uint64_t)ahi << 32) | alo));
    b = __longlong_as_double((long long)(((uint64_t)bhi << 32) | blo));
}

__device__ inline double row_sum(double v) {
    v += partner<0>(v);
    v += partner<1>(v);
    v += partner<2>(v);
    v += partner<3>(v);
    return v;
}

__device__ inline void wave_sum6(double x[6]) {
    double y[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double a = x[q], b = x[q + 3];
        swap_halves(a, b, false);
        y[q] = a + b;  // lanes 0-31: x[q] over lanes l, l+32; lanes 32-63: x[q+3]
    }
    double a = y[0], b = y[1];
    swap_halves(a, b, true);
    double z0 = row_sum(a + b);  // rows 0, 1, 2, 3: x0, x1, x3, x4
    a = y[2]; b = y[2];
    swap_halves(a, b, true);
    double z1 = row_sum(a + b);  // rows 0, 1: x2; rows 2, 3: x5
    x[0] = readlane(z0, 0);
    x[1] = readlane(z0, 16);
    x[3] = readlane(z0, 32);
    x[4] = readlane(z0, 48);
    x[2] = readlane(z1, 0);
    x[5] = readlane(z1, 32);
}

// Group totals of six compensated lane partials (see group_sum_comp).
template <int L, class T> __device__ inline void group_sum_comp6(const Comp<T> c[6], double out[6]) {
    if constexpr (L == 64 && ESBGK_COMP_BUTTERFLY == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) out[q] = (double)c[q].hi + (double)c[q].lo;
        wave_sum6(out);
    } else {
#pragma unroll
        for (int q = 0; q < 6; ++q) out[q] = group_sum_comp<L>(c[q]);
    }
}

// -------------------------------------------------------- kernel geometry

struct Geom {
    int nx, ny, nv, nv2;
    double dx, dy, dv, vmax, w;  // w = dv^2 quadrature weight
    double idx, idy;             // 1/dx, 1/dy
    double beta, tau, dt;
    int recon, correction;
};

// ------------------------------------------ per-cell Gaussian parameters
//
// A sampled Gaussian with the conservation correction is stored per cell as
// 16 doubles so that later kernels can re-evaluate it at any node without
// touching the velocity block:
//   Ghat(v) = exp2(qxx xi_x^2 + qxy xi_x xi_y + qyy xi_y^2) * (c . psi),
//   xi = v - u, psi = (1, a, b, a^2, a b, b^2), (a, b) = xi / sqrt(T),
// where the Gaussian's prefactor rho / (2 pi sqrt(det Tt)) is folded into c.
enum GP { GP_UX = 0, GP_UY, GP_QXX, GP_QXY, GP_QYY, GP_PREF, GP_IST, GP_C0, GP_C1, GP_C2,
          GP_C3, GP_C4, GP_C5, GP_RHO, GP_T, GP_PAD, GP_N };

// Exponent part of the Gaussian with density rho, mean u and covariance Tt
// (Sec. 2: rho / sqrt(det(2 pi Tt)) exp(-xi^T Tt^{-1} xi / 2)), FP64.
// c = pref * e0 (no correction yet).  Returns false if Tt is not SPD.
__device__ inline bool gauss_params(double rho, double ux, double uy, double T, double txx,
                                    double txy, double tyy, double *gp) {
    const double det = txx * tyy - txy * txy;
    const bool ok = det > 0.0 && txx > 0.0 && rho > 0.0 && T > 0.0;
    const double idet = 1.0 / det;
    gp[GP_UX] = ux;
    gp[GP_UY] = uy;
    gp[GP_QXX] = (-0.5 * kLog2e) * (tyy * idet);
    gp[GP_QXY] = kLog2e * (txy * idet);
    gp[GP_QYY] = (-0.5 * kLog2e) * (txx * idet);
    const double pref = rho / (2.0 * kPi * sqrt(det));
    gp[GP_PREF] = pref;
    gp[GP_IST] = 1.0 / sqrt(T);
    gp[GP_C0] = pref;
    gp[GP_C1] = gp[GP_C2] = gp[GP_C3] = gp[GP_C4] = gp[GP_C5] = 0.0;
    gp[GP_RHO] = rho;
    gp[GP_T] = T;
    gp[GP_PAD] = 0.0;
    return ok;
}

// Correction in deviation form, fast path.  r = t - (discrete moments of the
// sampled Gaussian up to order 2), scaled by 1/rho; solves M(Sigma) dc = r/rho
// with M the moment matrix of (1, a, b, a^2, ab, b^2) under the continuous
// Gaussian N(0, Sigma), Sigma = Tt/T: odd block Sigma itself, even block
// reduced to the covariance matrix of (a^2, ab, b^2) by eliminating dc0.  The
// discrete Gram matrix differs from M by the quadrature error, so the result
// leaves a residual of second order in that error.  All FP64.
__device__ inline void solve_correction_gaussian(const double rr[6], double sxx, double sxy, double syy,
                                                 double dc[6]) {
    const double ids = 1.0 / (sxx * syy - sxy * sxy);
    dc[1] = (syy * rr[1] - sxy * rr[2]) * ids;
    dc[2] = (sxx * rr[2] - sxy * rr[1]) * ids;
    // K d = rhs, K = Cov(a^2, ab, b^2)
    const double k11 = 2.0 * sxx * sxx, k12 = 2.0 * sxx * sxy, k13 = 2.0 * sxy * sxy;
    const double k22 = sxx * syy + sxy * sxy, k23 = 2.0 * sxy * syy, k33 = 2.0 * syy * syy;
    const double b1 = rr[3] - sxx * rr[0], b2 = rr[4] - sxy * rr[0], b3 = rr[5] - syy * rr[0];
    const double c11 = k22 * k33 - k23 * k23, c12 = k13 * k23 - k12 * k33, c13 = k12 * k23 - k13 * k22;
    const double c22 = k11 * k33 - k13 * k13, c23 = k12 * k13 - k11 * k23, c33 = k11 * k22 - k12 * k12;
    const double idet = 1.0 / (k11 * c11 + k12 * c12 + k13 * c13);
    dc[3] = (c11 * b1 + c12 * b2 + c13 * b3) * idet;
    dc[4] = (c12 * b1 + c22 * b2 + c23 * b3) * idet;
    dc[5] = (c13 * b1 + c23 * b2 + c33 * b3) * idet;
    dc[0] = rr[0] - (sxx * dc[3] + sxy * dc[4] + syy * dc[5]);
}

// Exact path: the discrete Gram matrix from the 15 moments S (of the scaled
// sampled Gaussian, order 00 10 01 20 11 02 30 21 12 03 40 31 22 13 04),
// A dc = r by Cholesky in FP64.  Returns false if A is not SPD.
__device__ inline bool solve_correction_gram(const double S[15], const double r[6], double dc[6]) {
    const int pp[6] = {0, 1, 0, 2, 1, 0}, qq[6] = {0, 0, 1, 0, 1, 2};
    double A[6][6];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int n = 0; n <= m; ++n) {
            const int p = pp[m] + pp[n], q = qq[m] + qq[n], d = p + q;
            A[m][n] = S[d * (d + 1) / 2 + q];
        }
    bool ok = true;
    double il[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
        ok = ok && d > 0.0;
        il[j] = 1.0 / sqrt(d);
#pragma unroll
        for (int i = j + 1; i < 6; ++i) {
            double s = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k];
            A[i][j] = s * il[j];
        }
    }
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = r[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= A[i][k] * y[k];
        y[i] = s * il[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= A[k][i] * dc[k];
        dc[i] = s * il[i];
    }
    return ok;
}

// Per-lane copy of a cell's Gaussian parameters in the arithmetic type, with
// the chunk-invariant parts of the exponent and the polynomial hoisted.
template <class T> struct GaussEval {
    T ux, uy, qxx, qxy, qyy, ist, c0, c1, c2, c3, c4, c5;
    __device__ inline void load(const double *gp) {
        ux = (T)gp[GP_UX]; uy = (T)gp[GP_UY];
        qxx = (T)gp[GP_QXX]; qxy = (T)gp[GP_QXY]; qyy = (T)gp[GP_QYY];
        ist = (T)gp[GP_IST];
        c0 = (T)gp[GP_C0]; c1 = (T)gp[GP_C1]; c2 = (T)gp[GP_C2];
        c3 = (T)gp[GP_C3]; c4 = (T)gp[GP_C4]; c5 = (T)gp[GP_C5];
    }
};

// Chunk-level constants of a Gaussian at y-velocity vy.
template <class T> struct GaussRow {
    T qy_lin, qy_const, p_lin, p_const;  // exponent = (qxx ex + qy_lin) ex + qy_const
    __device__ inline void set(const GaussEval<T> &g, T vy) {
        const T ey = vy - g.uy;
        const T b = ey * g.ist;
        qy_lin = g.qxy * ey;
        qy_const = g.qyy * ey * ey;
        p_lin = g.c1 + g.c4 * b;                   // poly = (c3 a + p_lin) a + p_const
        p_const = g.c0 + (g.c2 + g.c5 * b) * b;
    }
    // unscaled sampled Gaussian exp2(Q) at x-velocity vx
    __device__ inline T tilde(const GaussEval<T> &g, T vx) const {
        const T ex = vx - g.ux;
        return fast_exp2((g.qxx * ex + qy_lin) * ex + qy_const);
    }
    // the sampled Gaussian pref exp2(Q): one expression wherever it is formed,
    // so a value evaluated again equals the one staged
    __device__ inline T sampled(const GaussEval<T> &g, T pref, T vx) const { return pref * tilde(g, vx); }
    __device__ inline T hat(const GaussEval<T> &g, T vx) const {
        const T ex = vx - g.ux;
        const T a = ex * g.ist;
        return fast_exp2((g.qxx * ex + qy_lin) * ex + qy_const) * ((g.c3 * a + p_lin) * a + p_const);
    }
};

// error flag bits
enum { ERR_RHO = 1, ERR_T = 2, ERR_SPD = 4, ERR_NAN = 8 };

}  // namespace esbgk
