// kinetic_impl.h -- phase-space kernels of the kinetic IMEX stage (ES-BGK, 2D2V),
// instantiated per storage precision by kinetic_f64.hip, kinetic_f32.hip and
// kinetic_bf16.hip.
//
// stage_kernel fuses, for every kinetic cell (one L-lane group per cell):
//   transport L(f^(j)) of earlier stages at every node (upwind or minmod-limited
//     upwind flux, Sec. 3.2), read straight from the velocity-contiguous f arrays;
//   the explicit stage sum f* = f^n - dt sum_j At_ij L(f^(j)) + dt sum_j A_ij Q'_j
//     (eq. RKEI1).  With FP32 / FP64 stage arrays the implicit term of an
//     earlier stage j is taken as Q'_j = (f^(j) - f*_j) / (dt A_jj), which
//     equals (tau/eps)(Ghat_j - f^(j)) for the exact relaxation of stage j,
//     with f*_j = f^n - dt At_j1 L(f^n) rebuilt from the transport of f^n the
//     kernel forms anyway (no Gaussian is re-evaluated).  With BF16 stage
//     arrays that difference would carry their rounding at full weight, so
//     Ghat_j is re-evaluated from the per-cell parameters stage j stored;
//   the velocity moments of f* (rho, u, T, Theta; H3 and Sec. 2), with
//     compensated FP32 sums;
//   the FP64 closed form of the implicit relaxation,
//     Theta = (Theta* + lam (1-beta) T I) / (1 + lam (1-beta)),
//     Tt = (1-beta) T I + beta Theta, lam = dt A_ii tau/eps,
//     and the FP64 6x6 discrete-conservation correction of the sampled Gaussian;
//   f^(i) = (f* + lam Ghat) / (1 + lam), the single write of the stage.
// The last implicit stage of ARS(2,3,3) also writes the partial sum
//   P' = f^n - dt sum_j bt_j L(f^(j)) + dt sum_j b_j Q'_j   (j = 1 .. 3, L of f^(3) excluded),
// its own Q'_3 included once f^(3) is known.  The FINAL variant is the final
// combination (eq. RKEI2) f^{n+1} = P' - dt bt_3 L(f^(3)): it writes f^{n+1},
// its moments U^{n+1} and the L1 distance to the Maxwellian that the next
// regime update reads (eq. eqKintoFluid1).
#pragma once
#include <type_traits>

#include "kernels.h"

// implicit stages: stencil loads of the next work unit issued before the
// current one is computed
#ifndef ESBGK_PREFETCH
#define ESBGK_PREFETCH 1
#endif

// waves per SIMD the stage kernels are compiled for (caps their VGPR budget):
// implicit stages, final combination
#ifndef ESBGK_STAGE_MIN_WAVES
#define ESBGK_STAGE_MIN_WAVES 3
#endif
#ifndef ESBGK_FINAL_MIN_WAVES
#define ESBGK_FINAL_MIN_WAVES 4
#endif
// mixed form, first implicit stage: keep f^n at the cell in registers for the
// increment up to this many chunks per lane (else it is read again; measured
// faster at every instantiated size, 4 to 16 chunks)
#ifndef ESBGK_FNR_MAXC
#define ESBGK_FNR_MAXC 16
#endif


namespace esbgk {

__device__ inline int wrapi(int i, int n) { i %= n; return i < 0 ? i + n : i; }

struct Nbr {
    size_t c, xm1, xp1, xm2, xp2, ym1, yp1, ym2, yp2;  // cell * nv2
};

__device__ inline Nbr neighbours(int cell, const Geom &g) {
    const int i = cell % g.nx, j = cell / g.nx;
    const size_t n2 = (size_t)g.nv2;
    Nbr b;
    b.c = (size_t)cell * n2;
    b.xm1 = ((size_t)j * g.nx + wrapi(i - 1, g.nx)) * n2;
    b.xp1 = ((size_t)j * g.nx + wrapi(i + 1, g.nx)) * n2;
    b.xm2 = ((size_t)j * g.nx + wrapi(i - 2, g.nx)) * n2;
    b.xp2 = ((size_t)j * g.nx + wrapi(i + 2, g.nx)) * n2;
    b.ym1 = ((size_t)wrapi(j - 1, g.ny) * g.nx + i) * n2;
    b.yp1 = ((size_t)wrapi(j + 1, g.ny) * g.nx + i) * n2;
    b.ym2 = ((size_t)wrapi(j - 2, g.ny) * g.nx + i) * n2;
    b.yp2 = ((size_t)wrapi(j + 2, g.ny) * g.nx + i) * n2;
    return b;
}

// Upwind-mirrored limited difference: with g_{-2}, g_{-1}, g_0, g_1 the values
// ordered along the flow, (F_{+1/2} - F_{-1/2}) / |v| equals
//   q + (minmod(q, r) - minmod(p, q)) / 2,
//   p = g_{-1} - g_{-2}, q = g_0 - g_{-1}, r = g_1 - g_0.
template <class T> __device__ inline T limited_diff(T far, T up, T c, T dn) {
    const T p = up - far, q = c - up, r = dn - c;
    return q + (T)0.5 * (minmod(q, r) - minmod(p, q));
}

// Velocity bookkeeping of one chunk: first node k0, x-velocities of its 4
// nodes, its y-velocity.
template <class T> struct Chunk {
    int k0;
    bool active;
    bool xpos, ypos, straddle;  // upwind directions; straddle: v_x changes sign inside the chunk
    T vx[4], vy;
};

// Stencil values of one chunk of one f array: the cell's own values c, the
// y-neighbours upwind / downwind / far (y[0..2]) and the x-neighbours
// (x[0..2] upwind / downwind / far; a chunk that straddles v_x = 0 holds
// i-1, i+1, i-2, i+2 in x[0..3]).  RECON: 0 first-order upwind (only c, y[0],
// x[0] or x[0..1]), 1 minmod-limited upwind.
template <class T> struct Stencil {
    T c[4], y[3][4], x[4][4];
    T b[4];  // final combination: f^n at the cell, loaded with the chunk's first unit
};

// Issue the loads of a chunk's stencil.  The neighbour bases are wave-uniform
// when a wavefront owns one cell, so each load is a scalar base plus a 32-bit
// lane offset.
template <class S, int RECON>
__device__ inline void load_stencil(const S *f, const Nbr &nb, const Chunk<typename Storage<S>::T> &ch,
                                    Stencil<typename Storage<S>::T> &st) {
    const uint32_t k0 = (uint32_t)ch.k0;
    const bool ypos = ch.ypos;
    Storage<S>::load4(f + nb.c, k0, st.c);
    Storage<S>::load4(f + (ypos ? nb.ym1 : nb.yp1), k0, st.y[0]);
    if constexpr (RECON != 0) {
        Storage<S>::load4(f + (ypos ? nb.yp1 : nb.ym1), k0, st.y[1]);
        Storage<S>::load4(f + (ypos ? nb.ym2 : nb.yp2), k0, st.y[2]);
    }
    if (!ch.straddle) {
        const bool pos = ch.xpos;
        Storage<S>::load4(f + (pos ? nb.xm1 : nb.xp1), k0, st.x[0]);
        if constexpr (RECON != 0) {
            Storage<S>::load4(f + (pos ? nb.xp1 : nb.xm1), k0, st.x[1]);
            Storage<S>::load4(f + (pos ? nb.xm2 : nb.xp2), k0, st.x[2]);
        }
    } else {
        Storage<S>::load4(f + nb.xm1, k0, st.x[0]);
        Storage<S>::load4(f + nb.xp1, k0, st.x[1]);
        if constexpr (RECON != 0) {
            Storage<S>::load4(f + nb.xm2, k0, st.x[2]);
            Storage<S>::load4(f + nb.xp2, k0, st.x[3]);
        }
    }
}

// |v_x| (F_{i+1/2} - F_{i-1/2}) / dx + |v_y| (G_{j+1/2} - G_{j-1/2}) / dy at the
// 4 nodes of a chunk: the transport operator L of Sec. 3.2 with upwind or
// minmod-limited face values.
template <class T, int RECON>
__device__ inline void transport_of(const Stencil<T> &st, const Chunk<T> &ch, T idx, T idy, T out[4]) {
    const T avy = (ch.ypos ? ch.vy : -ch.vy) * idy;
    T Ly[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
        Ly[e] = avy * (RECON == 0 ? st.c[e] - st.y[0][e] : limited_diff(st.y[2][e], st.y[0][e], st.c[e], st.y[1][e]));
    if (!ch.straddle) {
        const bool pos = ch.xpos;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const T avx = (pos ? ch.vx[e] : -ch.vx[e]) * idx;
            out[e] = avx * (RECON == 0 ? st.c[e] - st.x[0][e]
                                       : limited_diff(st.x[2][e], st.x[0][e], st.c[e], st.x[1][e])) + Ly[e];
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool pos = ch.vx[e] > (T)0;
            const T avx = (pos ? ch.vx[e] : -ch.vx[e]) * idx;
            const T up = pos ? st.x[0][e] : st.x[1][e];
            if constexpr (RECON == 0) {
                out[e] = avx * (st.c[e] - up) + Ly[e];
            } else {
                const T far = pos ? st.x[2][e] : st.x[3][e];
                const T dn = pos ? st.x[1][e] : st.x[0][e];
                out[e] = avx * limited_diff(far, up, st.c[e], dn) + Ly[e];
            }
        }
    }
}

__device__ inline void raise_err(int *err, int bits, bool leader) {
    if (bits && leader) atomicOr(err, bits);
}

// XCD-aware work assignment: blocks are dealt to the 8 XCDs round-robin, so
// block b runs on XCD b % 8; each XCD gets a contiguous range of the cell list
// (contiguous list entries are spatially close cells that share halo data in
// that XCD's L2).  Returns the first list item of this block or -1.
__device__ inline int block_first_item(int count, int cells_per_block) {
    const int nblk = (count + cells_per_block - 1) / cells_per_block;
    const int per = (nblk + 7) / 8;
    const int b = blockIdx.x;
    const int xcd = b & 7, r = b >> 3;
    if (r >= per) return -1;
    const int first = (xcd * per + r) * cells_per_block;
    return first < count ? first : -1;
}

// Cell of this lane's group (-1 if the whole wavefront has no work).  Groups
// past the end of the list work on the last listed cell and store nothing, so
// that every lane takes part in the group-wide reductions.
struct GroupCell {
    int cell;
    bool valid;
};

template <int L, int WPB = 4> __device__ inline GroupCell group_cell(const int *list, int count) {
    constexpr int G = 64 / L;
    GroupCell gc{-1, false};
    const int first = block_first_item(count, WPB * G);
    if (first < 0) return gc;
    const int wave_first = first + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * G;
    if (wave_first >= count) return gc;
    if constexpr (L == 64) {
        // one cell per wavefront: keep its index (and all neighbour arithmetic) scalar
        gc.valid = true;
        gc.cell = __builtin_amdgcn_readfirstlane(list[wave_first]);
        return gc;
    }
    int item = wave_first + (int)((threadIdx.x & 63) / L);
    gc.valid = item < count;
    if (!gc.valid) item = count - 1;
    gc.cell = list[item];
    return gc;
}

// Chunk m of sub-lane s: chunk c = s + L m covers nodes 4c .. 4c+3 in
// row-major order (whole 128-byte rows per wave-wide load).  NV > 0 is the
// velocity grid size known at compile time: when L is a multiple of NV/4
// every lane keeps the same x-velocities in all its chunks and each chunk's
// y-row (hence its upwind direction) is a compile-time function of m, so
// neighbour selection and addressing fold into constants.  NV = 0 reads the
// size from g.
template <class T, int L, int NV>
__device__ inline Chunk<T> chunk_of(int s, int m, const Geom &g) {
    Chunk<T> ch;
    const int c = s + L * m;
    ch.k0 = 4 * c;
    const int nv = NV > 0 ? NV : g.nv;
    const int nq4 = nv >> 2;
    int ia, ib;
    if constexpr (NV > 0 && (L % (NV / 4)) == 0) {
        ia = 4 * (s % (NV / 4));
        ib = s / (NV / 4) + m * (L / (NV / 4));
        ch.active = ch.k0 < NV * NV;
    } else {
        ia = 4 * (c % nq4);
        ib = c / nq4;
        ch.active = ch.k0 < nv * nv;
    }
    const int half = nv >> 1;
    ch.xpos = ia >= half;
    ch.straddle = (NV > 0 && NV % 8 == 0) ? false : (ia < half && ia + 3 >= half);
    if constexpr (NV > 0 && (L % (NV / 4)) == 0 && ((NV / 2) % (L / (NV / 4))) == 0) {
        ch.ypos = m * (L / (NV / 4)) >= NV / 2;  // the rows of chunk slice m lie on one side
    } else {
        ch.ypos = ib >= half;
    }
    const T dv = (T)g.dv, v0 = (T)(-g.vmax + 0.5 * g.dv);
    ch.vy = v0 + (T)ib * dv;
#pragma unroll
    for (int e = 0; e < 4; ++e) ch.vx[e] = v0 + (T)(ia + e) * dv;
    return ch;
}

// Group-wide moments of the values v: compensated sums of f, v f and the raw
// second moments, centred in FP64.  out = {rho, ux, uy, T, Thxx, Thxy, Thyy}.
template <class T, int L, int C, int NV>
__device__ inline void group_moments(const T v[C][4], int s, const Geom &g, double out[7]) {
    Comp<T> cs[6];
    T part[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
        if (ch.active) {
            const T c0 = (v[m][0] + v[m][1]) + (v[m][2] + v[m][3]);
            const T cx = (ch.vx[0] * v[m][0] + ch.vx[1] * v[m][1]) + (ch.vx[2] * v[m][2] + ch.vx[3] * v[m][3]);
            const T cxx = (ch.vx[0] * ch.vx[0] * v[m][0] + ch.vx[1] * ch.vx[1] * v[m][1]) +
                          (ch.vx[2] * ch.vx[2] * v[m][2] + ch.vx[3] * ch.vx[3] * v[m][3]);
            part[0] += c0;
            part[1] += cx;
            part[2] += ch.vy * c0;
            part[3] += cxx;
            part[4] += ch.vy * cx;
            part[5] += ch.vy * ch.vy * c0;
        }
        if ((m & 3) == 3 || m == C - 1) {
#pragma unroll
            for (int q = 0; q < 6; ++q) { cs[q].add(part[q]); part[q] = 0; }
        }
    }
    double M[6];
    group_sum_comp6<L>(cs, M);
#pragma unroll
    for (int q = 0; q < 6; ++q) M[q] *= g.w;
    const double rho = M[0];
    const double irho = 1.0 / rho;
    const double ux = M[1] * irho, uy = M[2] * irho;
    const double pxx = M[3] - rho * ux * ux, pxy = M[4] - rho * ux * uy, pyy = M[5] - rho * uy * uy;
    out[0] = rho;
    out[1] = ux;
    out[2] = uy;
    out[3] = 0.5 * (pxx + pyy) * irho;
    out[4] = pxx * irho;
    out[5] = pxy * irho;
    out[6] = pyy * irho;
}

// L1 distance (eq. eqKintoFluid1) of the values v to the sampled Maxwellian
// with moments (rho, u, T), over the group's nodes.
template <class T, int L, int C, int NV>
__device__ inline double group_l1(const T v[C][4], int s, const Geom &g, double rho, double ux, double uy,
                                  double Tm) {
    const T pref = (T)(rho / (2.0 * kPi * Tm));
    const T qm = (T)(-0.5 * kLog2e / Tm);
    const T uxt = (T)ux, uyt = (T)uy;
    T l1 = 0;
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
        if (ch.active) {
            const T ey = ch.vy - uyt;
            const T qy = qm * ey * ey;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const T ex = ch.vx[e] - uxt;
                l1 += fabs(v[m][e] - pref * fast_exp2(qm * ex * ex + qy));
            }
        }
    }
    return g.w * (double)group_sum<L>(l1);
}

// Moment partial sums of one chunk of values v into part[6] (sum f, vx f,
// vy f, vx^2 f, vx vy f, vy^2 f), folded into the compensated lane sums every
// 4 chunks.
template <class T> struct MomentAcc {
    Comp<T> cs[6];
    T part[6] = {0, 0, 0, 0, 0, 0};
    __device__ inline void add(const Chunk<T> &ch, const T v[4]) {
        const T c0 = (v[0] + v[1]) + (v[2] + v[3]);
        const T cx = (ch.vx[0] * v[0] + ch.vx[1] * v[1]) + (ch.vx[2] * v[2] + ch.vx[3] * v[3]);
        const T cxx = (ch.vx[0] * ch.vx[0] * v[0] + ch.vx[1] * ch.vx[1] * v[1]) +
                      (ch.vx[2] * ch.vx[2] * v[2] + ch.vx[3] * ch.vx[3] * v[3]);
        part[0] += c0;
        part[1] += cx;
        part[2] += ch.vy * c0;
        part[3] += cxx;
        part[4] += ch.vy * cx;
        part[5] += ch.vy * ch.vy * c0;
    }
    __device__ inline void fold() {
#pragma unroll
        for (int q = 0; q < 6; ++q) { cs[q].add(part[q]); part[q] = 0; }
    }
    // {rho, ux, uy, T, Thxx, Thxy, Thyy} of the group
    template <int L> __device__ inline void finish(double w, double out[7]) {
        fold();
        double M[6];
        group_sum_comp6<L>(cs, M);
#pragma unroll
        for (int q = 0; q < 6; ++q) M[q] *= w;
        const double rho = M[0];
        const double irho = 1.0 / rho;
        const double ux = M[1] * irho, uy = M[2] * irho;
        const double pxx = M[3] - rho * ux * ux, pxy = M[4] - rho * ux * uy, pyy = M[5] - rho * uy * uy;
        out[0] = rho;
        out[1] = ux;
        out[2] = uy;
        out[3] = 0.5 * (pxx + pyy) * irho;
        out[4] = pxx * irho;
        out[5] = pxy * irho;
        out[6] = pyy * irho;
    }
};

// Per-lane staging in LDS between the passes over a cell's nodes: each lane
// writes and reads back only its own 16-byte (FP32) slots, so no barrier is
// needed.
//
// LDS of the stage kernels, per wave, in arrays of C x 64 x 4 values: f*
// (always); the sampled Gaussian of an implicit stage while the kernel's
// arrays for four waves fit in 80 KB (stage 2 up to nv = 48, the last stage of
// ARS(2,3,3) up to nv = 32, in FP32), else the relaxation evaluates it again,
// identically; and, in the last implicit stage of ARS(2,3,3), P until f^(3) is
// known, when it fits beside the others (else it goes to an FP32 buffer it is
// read back from; the lane reads its own write, from L2).  Four waves per
// block when the block's LDS stays within 80 KB, else one.  (Measured: at
// nv = 64 re-evaluating the Gaussian at higher occupancy is 18% faster than
// staging it; at nv = 48 staging is faster for stage 2, re-evaluating with P in
// LDS faster for the last stage.)
#ifndef ESBGK_P_LDS
#define ESBGK_P_LDS 1
#endif
#ifndef ESBGK_G_LDS
#define ESBGK_G_LDS 1
#endif
template <class T, int C> __host__ __device__ constexpr int lds_array_bytes() {
    return C * 64 * 4 * (int)sizeof(T);
}
template <class T, int C, bool KEEP_P> __host__ __device__ constexpr bool g_in_lds() {
    return ESBGK_G_LDS && 4 * (KEEP_P ? 3 : 2) * lds_array_bytes<T, C>() <= 80 * 1024;
}
template <class T, int C> __host__ __device__ constexpr bool p_in_lds() {
    return ESBGK_P_LDS && (2 + (g_in_lds<T, C, true>() ? 1 : 0)) * lds_array_bytes<T, C>() <= 80 * 1024;
}
// the side output P is held until the relaxation has added the stage's own Q'
template <bool SIDE> __host__ __device__ constexpr bool keep_p() { return SIDE; }
template <class T, int C, bool FINAL, bool KEEP_P> __host__ __device__ constexpr int stage_arrays() {
    return 1 + ((!FINAL && g_in_lds<T, C, KEEP_P>()) ? 1 : 0) + ((KEEP_P && p_in_lds<T, C>()) ? 1 : 0);
}
template <class T, int C, bool FINAL, bool KEEP_P> __host__ __device__ constexpr int stage_waves() {
    return 4 * stage_arrays<T, C, FINAL, KEEP_P>() * lds_array_bytes<T, C>() <= 80 * 1024 ? 4 : 1;
}

// Optional LDS arrays, as (possibly empty) bases so that an absent one takes no space.
template <class T, int W, int C, bool ON> struct LdsGauss { T g[W][C][64][4]; };  // sampled Gaussian
template <class T, int W, int C> struct LdsGauss<T, W, C, false> {};
template <class T, int W, int C, bool ON> struct LdsPartial { T p[W][C][64][4]; };  // P until f^(3) is known
template <class T, int W, int C> struct LdsPartial<T, W, C, false> {};

template <class T, int C, bool FINAL, bool KEEP_P>
struct StageLds : LdsGauss<T, stage_waves<T, C, FINAL, KEEP_P>(), C, !FINAL && g_in_lds<T, C, KEEP_P>()>,
                  LdsPartial<T, stage_waves<T, C, FINAL, KEEP_P>(), C, KEEP_P && p_in_lds<T, C>()> {
    static constexpr int W = stage_waves<T, C, FINAL, KEEP_P>();
    static constexpr bool P = KEEP_P && p_in_lds<T, C>();
    static constexpr bool G = !FINAL && g_in_lds<T, C, KEEP_P>();
    T v[W][C][64][4];  // [wave in block][chunk][lane][node]: f*
};

// The discrete-conservation correction of a sampled Gaussian (a reading: the
// paper states exact conservation, Sec. 3.6).  With xi = (v-u)/sqrt(T),
// psi = (1, a, b, a^2, ab, b^2), the corrected Gaussian is
//   Ghat = Gtilde (1 + dc . psi)
// with dc chosen so that Ghat's discrete moments of psi equal the continuous
// ones t = (rho, 0, 0, rho Tt/T).  Pass 1 (gaussian_pass) evaluates Gtilde at
// every node (into LDS when glds is given) and accumulates its six discrete
// moments of order <= 2 (compensated); r = t - those.  When |r|/rho is below
// tol the moment matrix is replaced by the continuous Gaussian's (closed form,
// residual second order in the quadrature error); otherwise the nine higher
// discrete moments are summed (from LDS, or over Gtilde evaluated again) and
// the exact discrete Gram matrix is solved.  Returns error bits.
template <class T, int L, int C, int NV>
__device__ inline int correction_coeffs(const T (*glds)[64][4], int s, int lane, const Geom &g,
                                        const GaussEval<T> &ge, T pref, const double Slow[6], double rho,
                                        double Tm, double txx, double txy, double tyy, double tol,
                                        double dc[6]) {
    const double iT = 1.0 / Tm;
    double r[6];
    r[0] = rho - Slow[0];
    r[1] = -Slow[1];
    r[2] = -Slow[2];
    r[3] = rho * txx * iT - Slow[3];
    r[4] = rho * txy * iT - Slow[4];
    r[5] = rho * tyy * iT - Slow[5];
    double rmax = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) rmax = fmax(rmax, fabs(r[q]));
    if (rmax <= tol * rho) {
        const double irho = 1.0 / rho;
        double rr[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) rr[q] = r[q] * irho;
        solve_correction_gaussian(rr, txx * iT, txy * iT, tyy * iT, dc);
        return 0;
    }
    // exact path: moments of order 3 and 4 of the sampled Gaussian (staged in
    // glds, or evaluated again)
    T high[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
        if (ch.active) {
            const T b = (ch.vy - ge.uy) * ge.ist;
            GaussRow<T> gr;
            if (!glds) gr.set(ge, ch.vy);
            T p[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const T G = glds ? glds[m][lane][e] : gr.sampled(ge, pref, ch.vx[e]);
                const T a = (ch.vx[e] - ge.ux) * ge.ist;
                const T Ga = G * a, Ga2 = Ga * a, Ga3 = Ga2 * a;
                p[0] += G; p[1] += Ga; p[2] += Ga2; p[3] += Ga3; p[4] += Ga3 * a;
            }
            const T b2 = b * b, b3 = b2 * b, b4 = b2 * b2;
            high[0] += p[3]; high[1] += b * p[2]; high[2] += b2 * p[1]; high[3] += b3 * p[0];
            high[4] += p[4]; high[5] += b * p[3]; high[6] += b2 * p[2]; high[7] += b3 * p[1];
            high[8] += b4 * p[0];
        }
    }
    double S[15];
#pragma unroll
    for (int q = 0; q < 6; ++q) S[q] = Slow[q];
#pragma unroll
    for (int q = 0; q < 9; ++q) S[6 + q] = g.w * (double)group_sum<L>(high[q]);
    return solve_correction_gram(S, r, dc) ? 0 : ERR_SPD;
}

// Pass 1 over the nodes for the Gaussian with parameters ge (prefactor pref):
// Gtilde into glds (when given), the six compensated discrete moments of order
// <= 2 into Slow, and (when vlds is given) v <- (v + lam Gtilde) * inv1 in place.
template <class T, int L, int C, int NV>
__device__ inline void gaussian_pass(T (*glds)[64][4], T (*vlds)[64][4], int s, int lane, const Geom &g,
                                     const GaussEval<T> &ge, T pref, T lam, T inv1, double Slow[6]) {
    Comp<T> lowc[6];
    T low[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
        if (ch.active) {
            GaussRow<T> gr;
            gr.set(ge, ch.vy);
            const T b = (ch.vy - ge.uy) * ge.ist;
            T p0 = 0, p1 = 0, p2 = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const T G = gr.sampled(ge, pref, ch.vx[e]);
                const T a = (ch.vx[e] - ge.ux) * ge.ist;
                const T Ga = G * a;
                p0 += G; p1 += Ga; p2 += Ga * a;
                if (glds) glds[m][lane][e] = G;
                if (vlds) vlds[m][lane][e] = (vlds[m][lane][e] + lam * G) * inv1;
            }
            low[0] += p0; low[1] += p1; low[2] += b * p0;
            low[3] += p2; low[4] += b * p1; low[5] += b * b * p0;
        }
        if ((m & 3) == 3 || m == C - 1) {
#pragma unroll
            for (int q = 0; q < 6; ++q) { lowc[q].add(low[q]); low[q] = 0; }
        }
    }
    group_sum_comp6<L>(lowc, Slow);
#pragma unroll
    for (int q = 0; q < 6; ++q) Slow[q] *= g.w;
}

// Tolerance on |r|/rho for the closed-form correction: its residual is about
// the square of the quadrature error, far below the arithmetic's rounding.
template <class T> __device__ constexpr double correction_tol() { return sizeof(T) == 8 ? 1e-9 : 1e-6; }

// Storage of the partial sum P of the final combination: at least FP32 (it is
// a state-like quantity, rounded into f^{n+1}).
template <class S> struct PartialOf { using type = S; };
template <> struct PartialOf<bf16_t> { using type = float; };

// Increment storage of the mixed form (FP32 state, 16-bit stage storage):
// each BF16 array holds a difference to an FP32 array that its reader reads at
// the same nodes anyway, so the rounding error is relative to an increment of
// one stage rather than to f, at the HBM traffic of plain BF16 stage arrays.
//   f^(2) is stored as f^(2) - f^n (stage 3 transports f^n at the same stencil);
//   stage 3 stores f^(3) in FP32 and the partial sum as P - f^(3) (the final
//   combination reads f^(3) at the stencil and P only at the cell).
// Buffer cells are filled to match (f^(2): Mhat(U) - f^n; f^(3): Mhat(U)).
template <class SN, class SS> __host__ __device__ constexpr bool increment_storage() {
    return !std::is_same<SN, SS>::value;
}

// dst += src over the stencil entries load_stencil fills for chunk ch.
template <class T, int RECON> __device__ inline void add_stencil(Stencil<T> &dst, const Stencil<T> &src,
                                                                const Chunk<T> &ch) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        dst.c[e] += src.c[e];
        dst.y[0][e] += src.y[0][e];
        dst.x[0][e] += src.x[0][e];
        if (RECON != 0) {
            dst.y[1][e] += src.y[1][e];
            dst.y[2][e] += src.y[2][e];
            dst.x[2][e] += src.x[2][e];
        }
        if (RECON != 0 || ch.straddle) dst.x[1][e] += src.x[1][e];
        if (RECON != 0 && ch.straddle) dst.x[3][e] += src.x[3][e];
    }
}

template <class SN, class SS, int NV, int L, int C, int NL, int NQ, bool FINAL, int RECON, bool SIDE>
__global__ __launch_bounds__((64 * stage_waves<typename Storage<SN>::T, C, FINAL, keep_p<SIDE>()>()),
                             (FINAL ? ESBGK_FINAL_MIN_WAVES : ESBGK_STAGE_MIN_WAVES)) void stage_kernel(
    StageArgs a) {
    using T = typename Storage<SN>::T;
    using SP = typename PartialOf<SN>::type;
    static_assert(std::is_same<T, typename Storage<SS>::T>::value, "one arithmetic type per kernel");
    constexpr bool INC = increment_storage<SN, SS>();
    static_assert(!INC || std::is_same<SP, T>::value, "increments are taken over state-precision arrays");
    static_assert(!INC || ESBGK_PREFETCH, "increment storage completes stencils in the prefetch buffer");
    constexpr bool KEEP_P = keep_p<SIDE>();
    using Lds = StageLds<T, C, FINAL, KEEP_P>;
    __shared__ Lds lds;
    const Geom &g = a.g;
    const GroupCell gc = group_cell<L, Lds::W>(a.list, *a.count);
    if (gc.cell < 0) return;
    const int cell = gc.cell;
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int s = lane & (L - 1);
    const bool leader = gc.valid && s == 0;
    const Nbr nb = neighbours(cell, g);
    const T idx = (T)g.idx, idy = (T)g.idy;
    const double te = g.tau / a.eps[cell];
    const T dt = (T)g.dt;
    // implicit term from the stage difference (FP32 / FP64 stage arrays) or
    // from the re-evaluated Gaussian (BF16 stage arrays)
    constexpr bool QDIFF = qdiff_form<SS>();
    GaussEval<T> gq;
    if constexpr (!QDIFF && NQ > 0) gq.load(a.pq + (size_t)cell * GP_N);

    // ---- explicit part of the stage, moments on the fly
    MomentAcc<T> macc;
    constexpr int NU = C * NL;
    constexpr bool PF = ESBGK_PREFETCH != 0;
    constexpr int NB = PF ? 2 : 1;
    T base[4], acc[4], qsum[4];  // base: f^n at the cell (final combination: the partial sum P)
    T pacc[4], psum[4];          // side output P of the last implicit stage
    T fsq[4];                    // f*_j of the stage whose implicit term enters: f^n - dt At_j1 L(f^n)
    // mixed form, first implicit stage: f^n at the cell, the reference of the
    // stored increment, kept in registers from the explicit pass
    constexpr bool FNR = INC && !SIDE && NL == 1 && C <= ESBGK_FNR_MAXC;
    T fnr[FNR ? C : 1][4];
    // Per-unit work once its transport Lt and centre values cc are known.
    auto unit_body = [&](int m, int l, const Chunk<T> &ch, const T Lt[4], const T cc[4]) {
        const T cl = (T)a.cl[l];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            acc[e] = l == 0 ? cl * Lt[e] : acc[e] + cl * Lt[e];
            if (l == 0) qsum[e] = 0;
        }
        if constexpr (SIDE) {
            const T sl = (T)a.scl[l];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                pacc[e] = l == 0 ? sl * Lt[e] : pacc[e] + sl * Lt[e];
                if (l == 0) psum[e] = 0;
            }
        }
        // implicit term of the stage whose state this unit transports:
        // dt A_ij Q'_j = (A_ij / A_jj)(f^(j) - f*_j), f*_j formed from L(f^n)
        static_assert(NQ == 0 || (NQ == 1 && NL == 2), "one implicit term, that of the stage after f^n");
        if constexpr (NQ > 0 && QDIFF) {
            if (l == 0) {
                const T tn = (T)a.ctn;
#pragma unroll
                for (int e = 0; e < 4; ++e) fsq[e] = base[e] - dt * (tn * Lt[e]);
            } else {
                const T cq = (T)(a.qa / a.qd);
                const T sq = SIDE ? (T)(a.qb / a.qd) : (T)0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T hm = cc[e] - fsq[e];
                    qsum[e] += cq * hm;
                    if (SIDE) psum[e] += sq * hm;
                }
            }
        } else if constexpr (NQ > 0) {
            if (l == 1) {
                GaussRow<T> gr;
                gr.set(gq, ch.vy);
                const T cq = (T)(a.qa * g.dt * te);
                const T sq = SIDE ? (T)(a.qb * g.dt * te) : (T)0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T hm = gr.hat(gq, ch.vx[e]) - cc[e];
                    qsum[e] += cq * hm;
                    if (SIDE) psum[e] += sq * hm;
                }
            }
        }
        if (l == NL - 1) {
            T fs[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) fs[e] = (base[e] - dt * acc[e]) + qsum[e];
            macc.add(ch, fs);
#pragma unroll
            for (int e = 0; e < 4; ++e) lds.v[wave][m][lane][e] = fs[e];
            if (FINAL && gc.valid) Storage<SN>::store4((SN *)a.fout + nb.c, (uint32_t)ch.k0, fs);
            if (SIDE && gc.valid) {
                // P = f^n - dt sum_j bt_j L(f^(j)) + dt sum_j b_j Q'_j over the stages so far
                T pv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) pv[e] = (base[e] - dt * pacc[e]) + psum[e];
                // held until the relaxation: in LDS, else in the FP32 buffer it is
                // read back from (the lane reads its own write)
                if constexpr (Lds::P) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) lds.p[wave][m][lane][e] = pv[e];
                } else if constexpr (INC) {
                    Storage<SP>::store4((SP *)a.fout + nb.c, (uint32_t)ch.k0, pv);
                } else {
                    Storage<SP>::store4((SP *)a.sout + nb.c, (uint32_t)ch.k0, pv);
                }
            }
        }
    };
    // Work unit u = (chunk m = u / NL, transported array l = u % NL); with
    // prefetching the loads of the next (half) unit are in flight while the
    // current one is computed.  The source arrays of the implicit terms are
    // the last NQ transported arrays (the launcher checks this), so their
    // values are the stencil centres.
    {
        Stencil<T> sb[NB];
        auto load_unit = [&](int u, int slot) {
            const int m = u / NL, l = u % NL;
            const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
            if (!ch.active) return;
            if (!FINAL && l == 0)
                load_stencil<SN, RECON>((const SN *)a.fl[0], nb, ch, sb[slot]);
            else if (FINAL && INC)
                load_stencil<SP, RECON>((const SP *)a.fl[0], nb, ch, sb[slot]);  // f^(3) in FP32
            else
                load_stencil<SS, RECON>((const SS *)a.fl[l], nb, ch, sb[slot]);
            if (FINAL && INC)
                Storage<SS>::load4((const SS *)a.fn + nb.c, (uint32_t)ch.k0, sb[slot].b);  // P - f^(3)
            else if (FINAL)
                Storage<SP>::load4((const SP *)a.fn + nb.c, (uint32_t)ch.k0, sb[slot].b);
        };
        // Increment storage, stage 3: the loaded f^(2) - f^n of unit u (its
        // chunk's second unit) plus f^n, the stencil of the unit before.
        auto complete_unit = [&](int u) {
            if constexpr (INC && !FINAL) {
                const int m = u / NL, l = u % NL;
                const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
                if (ch.active && l == 1) add_stencil<T, RECON>(sb[u & 1], sb[(u - 1) & 1], ch);
            }
        };
        if (PF) load_unit(0, 0);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int m = u / NL, l = u % NL;
            const int slot = PF ? (u & 1) : 0;
            const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
            if (PF) {
                if (u + 1 < NU) load_unit(u + 1, (u + 1) & 1);
            } else {
                load_unit(u, 0);
            }
            const Stencil<T> &cur = sb[slot];
            if (ch.active) {
                if (l == 0) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)  // stages transport f^n first; the final combination's base is P
                        base[e] = !FINAL ? cur.c[e] : INC ? cur.c[e] + cur.b[e] : cur.b[e];
                    if constexpr (FNR) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) fnr[m][e] = base[e];
                    }
                }
                T Lt[4];
                transport_of<T, RECON>(cur, ch, idx, idy, Lt);
                unit_body(m, l, ch, Lt, cur.c);
            }
            if (INC && !FINAL && u + 1 < NU) complete_unit(u + 1);
            if (l == NL - 1 && (m & 3) == 3) macc.fold();
            // bounded register use: at most two units' loads live at a time
            __builtin_amdgcn_sched_barrier(0);
        }
    }

    // ---- moments of f*
    double mo[7];
    macc.template finish<L>(g.w, mo);
    const double rho = mo[0], ux = mo[1], uy = mo[2], Tm = mo[3];
    int errbits = 0;
    if (!(rho > 0.0)) errbits |= ERR_RHO;
    if (!(Tm > 0.0)) errbits |= ERR_T;
    if (rho != rho || Tm != Tm) errbits |= ERR_NAN;

    // L1 distance to the Maxwellian of (rho, u, T) (the relaxation keeps them)
    const bool want_l1 = FINAL || a.emit;
    const T mpref = (T)(rho / (2.0 * kPi * Tm)), mq = (T)(-0.5 * kLog2e / Tm);
    const T uxt = (T)ux, uyt = (T)uy;
    T l1 = 0;

    if constexpr (!FINAL) {
        // ---- FP64 closed form of the implicit relaxation
        const double lam = g.dt * a.aii * te;
        const double beta = g.beta;
        const double k = lam * (1.0 - beta);
        const double ik = 1.0 / (1.0 + k);
        const double txx = (1.0 - beta) * Tm + beta * ((mo[4] + k * Tm) * ik);
        const double txy = beta * (mo[5] * ik);
        const double tyy = (1.0 - beta) * Tm + beta * ((mo[6] + k * Tm) * ik);
        double gp[GP_N];
        if (!gauss_params(rho, ux, uy, Tm, txx, txy, tyy, gp)) errbits |= ERR_SPD;
        GaussEval<T> ge;
        ge.load(gp);
        const T lamt = (T)lam, inv1 = (T)(1.0 / (1.0 + lam));
        // ---- Gaussian pass: Gtilde into LDS and its low-order discrete moments
        double Slow[6];
        T(*gl)[64][4] = nullptr;
        if constexpr (Lds::G) gl = lds.g[wave];
        const T prefg = (T)gp[GP_PREF];
        gaussian_pass<T, L, C, NV>(gl, nullptr, s, lane, g, ge, prefg, lamt, inv1, Slow);
        double dc[6] = {0, 0, 0, 0, 0, 0};
        if (g.correction)
            errbits |= correction_coeffs<T, L, C, NV>(gl, s, lane, g, ge, prefg, Slow, rho, Tm, txx, txy, tyy,
                                                      correction_tol<T>(), dc);
        if (!QDIFF && a.pout && leader) {
            // per-cell parameters of the corrected Gaussian, for the next stage's implicit term
            const double pref = gp[GP_PREF];
            double *o = a.pout + (size_t)cell * GP_N;
#pragma unroll
            for (int q = 0; q < GP_N; ++q)
                o[q] = (q >= GP_C0 && q < GP_C0 + 6) ? pref * ((q == GP_C0 ? 1.0 : 0.0) + dc[q - GP_C0]) : gp[q];
        }

        // ---- relaxation: f = (f* + lam Gtilde (1 + dc . psi)) / (1 + lam), the stage's single write
        const T d0 = (T)dc[0], d1 = (T)dc[1], d2 = (T)dc[2], d3 = (T)dc[3], d4 = (T)dc[4], d5 = (T)dc[5];
        // side output: P' = P + dt b_i Q'_i = P + (b_i / A_ii)(f^(i) - f*_i)
        const T sfin = SIDE ? (T)a.sfin : (T)0;
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
            if (ch.active) {
                const T b = (ch.vy - ge.uy) * ge.ist;
                const T plin = d1 + d4 * b, pconst = d0 + (d2 + d5 * b) * b;
                GaussRow<T> gr;
                if (!Lds::G) gr.set(ge, ch.vy);
                // P held from the explicit pass (side output), or the mixed form's
                // reference of the stored increment of stage 2 (f^n)
                T rv[4] = {0, 0, 0, 0};
                if constexpr (Lds::P) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) rv[e] = lds.p[wave][m][lane][e];
                } else if constexpr (KEEP_P && INC) {
                    Storage<SP>::load4((const SP *)a.fout + nb.c, (uint32_t)ch.k0, rv);
                } else if constexpr (KEEP_P) {
                    Storage<SP>::load4((const SP *)a.sout + nb.c, (uint32_t)ch.k0, rv);
                } else if constexpr (FNR) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) rv[e] = fnr[m][e];
                } else if constexpr (INC) {
                    Storage<SN>::load4((const SN *)a.fn + nb.c, (uint32_t)ch.k0, rv);
                }
                T fv[4], sv[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T aa = (ch.vx[e] - ge.ux) * ge.ist;
                    T Gt;
                    if constexpr (Lds::G) Gt = lds.g[wave][m][lane][e];
                    else Gt = gr.sampled(ge, prefg, ch.vx[e]);
                    const T Ghat = Gt * ((T)1 + ((d3 * aa + plin) * aa + pconst));
                    const T fs = lds.v[wave][m][lane][e];
                    fv[e] = (fs + lamt * Ghat) * inv1;
                    if constexpr (KEEP_P) {
                        const T pn = rv[e] + sfin * (fv[e] - fs);
                        sv[e] = INC ? pn - fv[e] : pn;
                    } else {
                        sv[e] = INC ? fv[e] - rv[e] : fv[e];
                    }
                }
                if (gc.valid) {
                    if constexpr (KEEP_P && INC) {
                        Storage<SP>::store4((SP *)a.fout + nb.c, (uint32_t)ch.k0, fv);   // f^(3)
                        Storage<SS>::store4((SS *)a.sout + nb.c, (uint32_t)ch.k0, sv);   // P' - f^(3)
                    } else if constexpr (KEEP_P) {
                        Storage<SS>::store4((SS *)a.fout + nb.c, (uint32_t)ch.k0, fv);   // f^(3)
                        Storage<SP>::store4((SP *)a.sout + nb.c, (uint32_t)ch.k0, sv);   // P'
                    } else {
                        Storage<SS>::store4((SS *)a.fout + nb.c, (uint32_t)ch.k0, sv);
                    }
                }
                if (want_l1) {
                    const T ey = ch.vy - uyt, qy = mq * ey * ey;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const T ex = ch.vx[e] - uxt;
                        l1 += fabs(fv[e] - mpref * fast_exp2(mq * ex * ex + qy));
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
            if (ch.active) {
                const T ey = ch.vy - uyt, qy = mq * ey * ey;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T ex = ch.vx[e] - uxt;
                    l1 += fabs(lds.v[wave][m][lane][e] - mpref * fast_exp2(mq * ex * ex + qy));
                }
            }
        }
    }
    if (want_l1) {
        const double L1 = g.w * (double)group_sum<L>(l1);
        if (leader) a.l1out[cell] = L1;
    }
    if (leader) {
        const size_t nc = (size_t)a.nc;
        a.Uout[cell] = rho;
        a.Uout[nc + cell] = rho * ux;
        a.Uout[2 * nc + cell] = rho * uy;
        a.Uout[3 * nc + cell] = 0.5 * rho * (ux * ux + uy * uy) + rho * Tm;
    }
    raise_err(a.err, errbits, leader);
}

// ---------------------------------------------------------------- fills

// f = Mhat(U) at the listed cells (eq. Coupling_FluKin): the corrected sampled
// Maxwellian, i.e. the corrected Gaussian with Tt = T I.
#ifndef ESBGK_FILL_G_LDS
#define ESBGK_FILL_G_LDS 1
#endif
// The fill stages the sampled Gaussian in LDS while one array of four waves
// fits in 40 KB, else evaluates it again for the store.
template <class T, int C> __host__ __device__ constexpr bool fill_g_lds() {
    return ESBGK_FILL_G_LDS && 4 * lds_array_bytes<T, C>() <= 40 * 1024;
}
template <class T, int C> __host__ __device__ constexpr int fill_waves() {
    return (!fill_g_lds<T, C>() || 4 * lds_array_bytes<T, C>() <= 80 * 1024) ? 4 : 1;
}
template <class T, int W, int C, bool ON> struct FillLds { T g[W][C][64][4]; };
template <class T, int W, int C> struct FillLds<T, W, C, false> {};

template <class S, int NV, int L, int C>
__global__ __launch_bounds__((64 * fill_waves<typename Storage<S>::T, C>())) void fill_maxwellian_kernel(
    FillArgs<S> a) {
    using T = typename Storage<S>::T;
    constexpr int W = fill_waves<T, C>();
    constexpr bool GL = fill_g_lds<T, C>();
    __shared__ FillLds<T, W, C, GL> lds;
    const Geom &g = a.g;
    const GroupCell gc = group_cell<L, W>(a.list, *a.count);
    if (gc.cell < 0) return;
    const int cell = gc.cell;
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int s = lane & (L - 1);
    const size_t nc = (size_t)a.nc;
    const double rho = a.U[cell];
    const double ux = a.U[nc + cell] / rho, uy = a.U[2 * nc + cell] / rho;
    const double Tm = (a.U[3 * nc + cell] - 0.5 * rho * (ux * ux + uy * uy)) / rho;
    int errbits = 0;
    double gp[GP_N];
    if (!gauss_params(rho, ux, uy, Tm, Tm, 0.0, Tm, gp)) errbits |= ERR_SPD;
    GaussEval<T> ge;
    ge.load(gp);
    double Slow[6];
    T(*gl)[64][4] = nullptr;
    if constexpr (GL) gl = lds.g[wave];
    const T prefg = (T)gp[GP_PREF];
    gaussian_pass<T, L, C, NV>(gl, nullptr, s, lane, g, ge, prefg, (T)0, (T)1, Slow);
    double dc[6] = {0, 0, 0, 0, 0, 0};
    if (g.correction)
        errbits |= correction_coeffs<T, L, C, NV>(gl, s, lane, g, ge, prefg, Slow, rho, Tm, Tm, 0.0, Tm,
                                                  correction_tol<T>(), dc);
    const T d0 = (T)dc[0], d1 = (T)dc[1], d2 = (T)dc[2], d3 = (T)dc[3], d4 = (T)dc[4], d5 = (T)dc[5];
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
        if (ch.active && gc.valid) {
            const T b = (ch.vy - ge.uy) * ge.ist;
            const T plin = d1 + d4 * b, pconst = d0 + (d2 + d5 * b) * b;
            GaussRow<T> gr;
            if (!GL) gr.set(ge, ch.vy);
            T v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const T aa = (ch.vx[e] - ge.ux) * ge.ist;
                T G;
                if constexpr (GL) G = lds.g[wave][m][lane][e];
                else G = gr.sampled(ge, prefg, ch.vx[e]);
                v[e] = G + G * ((d3 * aa + plin) * aa + pconst);
            }
            if constexpr (std::is_same<S, bf16_t>::value) {
                // increment storage of a stage array (see increment_storage)
                if (a.ref_in) {
                    T r[4];
                    Storage<float>::load4(a.ref_in + (size_t)cell * g.nv2, (uint32_t)ch.k0, r);
#pragma unroll
                    for (int e = 0; e < 4; ++e) v[e] -= r[e];
                }
            }
            Storage<S>::store4(a.f + (size_t)cell * g.nv2, (uint32_t)ch.k0, v);
        }
    }
    raise_err(a.err, errbits, gc.valid && s == 0);
}

// U = moments(f) and the L1 distance at the listed cells (eq. Coupling_KinFlu,
// eq. eqKintoFluid1).
template <class S, int NV, int L, int C>
__global__ __launch_bounds__(256) void moments_kernel(MomArgs<S> a) {
    using T = typename Storage<S>::T;
    const Geom &g = a.g;
    const GroupCell gc = group_cell<L>(a.list, *a.count);
    if (gc.cell < 0) return;
    const int cell = gc.cell;
    const int s = (int)(threadIdx.x & (L - 1));
    T fv[C][4];
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const Chunk<T> ch = chunk_of<T, L, NV>(s, m, g);
#pragma unroll
        for (int e = 0; e < 4; ++e) fv[m][e] = 0;
        if (ch.active) Storage<S>::load4(a.f + (size_t)cell * g.nv2, (uint32_t)ch.k0, fv[m]);
    }
    double mo[7];
    group_moments<T, L, C, NV>(fv, s, g, mo);
    const double rho = mo[0], ux = mo[1], uy = mo[2], Tm = mo[3];
    const double L1 = group_l1<T, L, C, NV>(fv, s, g, rho, ux, uy, Tm);
    int errbits = 0;
    if (!(rho > 0.0)) errbits |= ERR_RHO;
    if (!(Tm > 0.0)) errbits |= ERR_T;
    const bool leader = gc.valid && s == 0;
    if (leader) {
        const size_t nc = (size_t)a.nc;
        a.U[cell] = rho;
        a.U[nc + cell] = rho * ux;
        a.U[2 * nc + cell] = rho * uy;
        a.U[3 * nc + cell] = 0.5 * rho * (ux * ux + uy * uy) + rho * Tm;
        if (a.l1) a.l1[cell] = L1;
    }
    raise_err(a.err, errbits, leader);
}

// ------------------------------------------------------- conversions

template <class S>
__global__ void f_from_f64_kernel(const double *in, S *out, size_t n4) {
    using T = typename Storage<S>::T;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n4; q += (size_t)gridDim.x * blockDim.x) {
        T v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (T)in[4 * q + e];
        Storage<S>::store4(out, 4 * q, v);
    }
}

template <class S>
__global__ void f_to_f64_kernel(const S *in, double *out, size_t n4) {
    using T = typename Storage<S>::T;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n4; q += (size_t)gridDim.x * blockDim.x) {
        T v[4];
        Storage<S>::load4(in, 4 * q, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) out[4 * q + e] = (double)v[e];
    }
}

// ------------------------------------------------------- host launchers

// Lanes per cell (L) and chunks of 4 nodes per lane (C) for a velocity grid:
// a 16-lane DPP row per cell (4 cells per wavefront) for up to 256 nodes, a
// 32-lane half-wavefront per cell up to 1024 nodes, a whole wavefront beyond.
struct Shape { int L, C; };

static inline Shape shape_for(int nv2) {
    const int chunks = nv2 / 4;
    if (chunks <= 64) return {16, 4};
    if (chunks <= 128) return {16, 8};
    if (chunks <= 256) return {32, 8};
    if (chunks <= 576) return {64, 9};
    return {64, 16};
}

static inline unsigned grid_for(int nmax, int cells_per_block) {
    const int nblk = (nmax + cells_per_block - 1) / cells_per_block;
    const int per = (nblk + 7) / 8;
    return (unsigned)(per > 0 ? per * 8 : 8);
}

// Velocity-grid sizes with compile-time instantiations (NV, L, C); any other
// multiple of 4 runs the NV = 0 kernels with the shape of shape_for().
// nv = 32: one cell per wavefront (neighbour bases and Gaussian parameters are
// wave-uniform) measured fastest against 2 cells (32 lanes) and 4 cells (16).
#ifndef ESBGK_NV32_L
#define ESBGK_NV32_L 64
#define ESBGK_NV32_C 4
#endif
#define ESBGK_STATIC_NV(X) X(16, 16, 4) X(32, ESBGK_NV32_L, ESBGK_NV32_C) X(48, 64, 9) X(64, 64, 16)
#define ESBGK_SHAPES(X) X(0, 16, 4) X(0, 16, 8) X(0, 32, 8) X(0, 64, 9) X(0, 64, 16)

template <class SN, class SS, int NL, int NQ, bool FINAL, bool SIDE>
static hipError_t stage_dispatch(const StageArgs &a, int nmax, hipStream_t st) {
    const Shape sh = shape_for(a.g.nv2);
#define ESBGK_CASE(NN, LL, CC)                                                                                     \
    if ((NN == 0) ? (sh.L == LL && sh.C == CC) : (a.g.nv == NN)) {                                                    \
        constexpr int WPB = stage_waves<typename Storage<SN>::T, CC, FINAL, keep_p<SIDE>()>();                      \
        const dim3 grid(grid_for(nmax, WPB * (64 / LL))), block(64 * WPB);                                          \
        if (a.g.recon == 0)                                                                                         \
            hipLaunchKernelGGL((stage_kernel<SN, SS, NN, LL, CC, NL, NQ, FINAL, 0, SIDE>), grid, block, 0, st, a);  \
        else                                                                                                        \
            hipLaunchKernelGGL((stage_kernel<SN, SS, NN, LL, CC, NL, NQ, FINAL, 1, SIDE>), grid, block, 0, st, a);  \
        return hipGetLastError();                                                                                   \
    }
    ESBGK_STATIC_NV(ESBGK_CASE)
    ESBGK_SHAPES(ESBGK_CASE)
#undef ESBGK_CASE
    return hipErrorInvalidValue;
}

template <class SN, class SS>
hipError_t launch_stage(const StageArgs &a, int nmax, hipStream_t st) {
    // the kernels take the implicit terms' states from the last NQ transported arrays
    for (int q = 0; q < a.nq; ++q)
        if (a.nl - a.nq + q < 0 || a.fq[q] != a.fl[a.nl - a.nq + q]) return hipErrorInvalidValue;
    if (a.sout && !(a.aii > 0.0)) return hipErrorInvalidValue;
    if (a.aii > 0.0) {
        if (a.nl < 1 || a.fl[0] != a.fn) return hipErrorInvalidValue;  // implicit stages transport f^n first
        // increment storage: the increment of the second implicit stage is taken over the partial sum
        if (increment_storage<SN, SS>() && a.nl == 2 && !a.sout) return hipErrorInvalidValue;
        if (a.nl == 1 && a.nq == 0 && !a.sout) return stage_dispatch<SN, SS, 1, 0, false, false>(a, nmax, st);
        if (a.nl == 2 && a.nq == 1 && !a.sout) return stage_dispatch<SN, SS, 2, 1, false, false>(a, nmax, st);
        if (a.nl == 2 && a.nq == 1 && a.sout) return stage_dispatch<SN, SS, 2, 1, false, true>(a, nmax, st);
    } else {
        // final combination from the partial sum P' of the last implicit stage
        if (a.nl == 1 && a.nq == 0) return stage_dispatch<SN, SS, 1, 0, true, false>(a, nmax, st);
    }
    return hipErrorInvalidValue;
}

template <class S>
hipError_t launch_fill(const FillArgs<S> &a, int nmax, hipStream_t st) {
    const Shape sh = shape_for(a.g.nv2);
#define ESBGK_CASE(NN, LL, CC)                                                                               \
    if ((NN == 0) ? (sh.L == LL && sh.C == CC) : (a.g.nv == NN)) {                                              \
        constexpr int WPB = fill_waves<typename Storage<S>::T, CC>();                                         \
        hipLaunchKernelGGL((fill_maxwellian_kernel<S, NN, LL, CC>), dim3(grid_for(nmax, WPB * (64 / LL))),    \
                           dim3(64 * WPB), 0, st, a);                                                         \
        return hipGetLastError();                                                                             \
    }
    ESBGK_STATIC_NV(ESBGK_CASE)
    ESBGK_SHAPES(ESBGK_CASE)
#undef ESBGK_CASE
    return hipErrorInvalidValue;
}

template <class S>
hipError_t launch_moments(const MomArgs<S> &a, int nmax, hipStream_t st) {
    const Shape sh = shape_for(a.g.nv2);
#define ESBGK_CASE(NN, LL, CC)                                                                       \
    if ((NN == 0) ? (sh.L == LL && sh.C == CC) : (a.g.nv == NN)) {                                      \
        hipLaunchKernelGGL((moments_kernel<S, NN, LL, CC>), dim3(grid_for(nmax, 4 * (64 / LL))),      \
                           dim3(256), 0, st, a);                                                      \
        return hipGetLastError();                                                                     \
    }
    ESBGK_STATIC_NV(ESBGK_CASE)
    ESBGK_SHAPES(ESBGK_CASE)
#undef ESBGK_CASE
    return hipErrorInvalidValue;
}

template <class S>
hipError_t launch_from_f64(const double *in, void *out, size_t n, hipStream_t st) {
    const size_t n4 = n / 4;
    unsigned grid = (unsigned)((n4 + 255) / 256 < 65536 ? (n4 + 255) / 256 : 65536);
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL((f_from_f64_kernel<S>), dim3(grid), dim3(256), 0, st, in, (S *)out, n4);
    return hipGetLastError();
}

template <class S>
hipError_t launch_to_f64(const void *in, double *out, size_t n, hipStream_t st) {
    const size_t n4 = n / 4;
    unsigned grid = (unsigned)((n4 + 255) / 256 < 65536 ? (n4 + 255) / 256 : 65536);
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL((f_to_f64_kernel<S>), dim3(grid), dim3(256), 0, st, (const S *)in, out, n4);
    return hipGetLastError();
}

#define ESBGK_INST_STAGE(SN, SS) template hipError_t launch_stage<SN, SS>(const StageArgs &, int, hipStream_t);
#define ESBGK_INST(S)                                                                        \
    ESBGK_INST_STAGE(S, S)                                                                   \
    template hipError_t launch_fill<S>(const FillArgs<S> &, int, hipStream_t);               \
    template hipError_t launch_moments<S>(const MomArgs<S> &, int, hipStream_t);             \
    template hipError_t launch_from_f64<S>(const double *, void *, size_t, hipStream_t);     \
    template hipError_t launch_to_f64<S>(const void *, double *, size_t, hipStream_t);

}  // namespace esbgk
