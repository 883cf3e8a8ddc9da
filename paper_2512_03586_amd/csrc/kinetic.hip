// kinetic.hip -- phase-space kernels of the kinetic IMEX stage (ES-BGK, 2D2V).
//
// stage_kernel fuses, for one kinetic cell per wavefront:
//   transport L(f^(j)) of earlier stages at every node (upwind or minmod-limited
//     upwind flux, Sec. 3.2), read straight from the velocity-contiguous f arrays;
//   the explicit stage sum f* = f^n - dt sum_j At_ij L(f^(j))
//     + dt sum_j A_ij (tau/eps)(Ghat_j - f^(j)) (eq. RKEI1), where Ghat_j is
//     re-evaluated from the per-cell parameters stage j stored;
//   the velocity moments of f* (rho, u, T, Theta; H3 and Sec. 2), compensated;
//   the FP64 closed form of the implicit relaxation,
//     Theta = (Theta* + lam (1-beta) T I) / (1 + lam (1-beta)),
//     Tt = (1-beta) T I + beta Theta, lam = dt A_ii tau/eps,
//     and the 6x6 discrete-conservation correction of the sampled Gaussian;
//   f^(i) = (f* + lam Ghat) / (1 + lam), the single write of the stage.
// With aii = 0 the same kernel is the final combination (eq. RKEI2): it writes
// f^{n+1}, its moments U^{n+1} and the L1 distance to the Maxwellian used by the
// next regime update (eq. eqKintoFluid1).
#include "kernels.h"

namespace esbgk {

__device__ inline int wrapi(int i, int n) { i %= n; return i < 0 ? i + n : i; }

struct Nbr {
    size_t c, xm1, xp1, xm2, xp2, ym1, yp1, ym2, yp2;  // cell * nv2
};

__device__ inline Nbr neighbours(int cell, const Geom &g) {
    int i = cell % g.nx, j = cell / g.nx;
    size_t n2 = (size_t)g.nv2;
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
// ordered along the flow, |v| (F_{+1/2} - F_{-1/2}) / h equals
//   |v| (q + (minmod(q, r) - minmod(p, q)) / 2) / h,
//   p = g_{-1} - g_{-2}, q = g_0 - g_{-1}, r = g_1 - g_0.
template <class T> __device__ inline T limited_diff(T far, T up, T c, T dn) {
    T p = up - far, q = c - up, r = dn - c;
    return q + (T)0.5 * (minmod(q, r) - minmod(p, q));
}

// L(f) at the 4 nodes of one chunk.
template <class S>
__device__ inline void transport4(const S *f, const Nbr &nb, int k0, const typename Storage<S>::T vx[4],
                                  typename Storage<S>::T vy, typename Storage<S>::T idx,
                                  typename Storage<S>::T idy, int recon, typename Storage<S>::T out[4]) {
    using T = typename Storage<S>::T;
    T fc[4], xm1[4], xp1[4];
    Storage<S>::load4(f, nb.c + k0, fc);
    const bool anypos = vx[3] > (T)0, anyneg = vx[0] < (T)0;
    const bool ypos = vy > (T)0;
    const size_t yup = ypos ? nb.ym1 : nb.yp1;
    const size_t ydn = ypos ? nb.yp1 : nb.ym1;
    const size_t yfar = ypos ? nb.ym2 : nb.yp2;
    const T avy = ypos ? vy : -vy;
    T yu[4];
    Storage<S>::load4(f, yup + k0, yu);
#pragma unroll
    for (int e = 0; e < 4; ++e) { xm1[e] = 0; xp1[e] = 0; }
    if (recon == 0) {
        if (anypos) Storage<S>::load4(f, nb.xm1 + k0, xm1);
        if (anyneg) Storage<S>::load4(f, nb.xp1 + k0, xp1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool pos = vx[e] > (T)0;
            T up = pos ? xm1[e] : xp1[e];
            T avx = pos ? vx[e] : -vx[e];
            out[e] = avx * (fc[e] - up) * idx + avy * (fc[e] - yu[e]) * idy;
        }
    } else {
        T xm2[4], xp2[4], yd[4], yf[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) { xm2[e] = 0; xp2[e] = 0; }
        Storage<S>::load4(f, nb.xm1 + k0, xm1);
        Storage<S>::load4(f, nb.xp1 + k0, xp1);
        if (anypos) Storage<S>::load4(f, nb.xm2 + k0, xm2);
        if (anyneg) Storage<S>::load4(f, nb.xp2 + k0, xp2);
        Storage<S>::load4(f, ydn + k0, yd);
        Storage<S>::load4(f, yfar + k0, yf);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool pos = vx[e] > (T)0;
            T far = pos ? xm2[e] : xp2[e];
            T up = pos ? xm1[e] : xp1[e];
            T dn = pos ? xp1[e] : xm1[e];
            T avx = pos ? vx[e] : -vx[e];
            out[e] = avx * limited_diff(far, up, fc[e], dn) * idx +
                     avy * limited_diff(yf[e], yu[e], fc[e], yd[e]) * idy;
        }
    }
}

__device__ inline void raise_err(int *err, int bits) {
    if (bits && (threadIdx.x & 63) == 0) atomicOr(err, bits);
}

// XCD-aware work assignment: blocks are dealt to the 8 XCDs round-robin, so
// block b runs on XCD b % 8; give each XCD a contiguous range of the cell list
// (contiguous cells share halo data in that XCD's L2).
__device__ inline int logical_item(int count, int waves_per_block) {
    int nblk = (count + waves_per_block - 1) / waves_per_block;
    int per = (nblk + 7) / 8;
    int b = blockIdx.x;
    int xcd = b & 7, r = b >> 3;
    if (r >= per) return -1;
    int lb = xcd * per + r;
    int item = lb * waves_per_block + (threadIdx.x >> 6);
    return item < count ? item : -1;
}

template <class S, int C>
__global__ __launch_bounds__(256) void stage_kernel(StageArgs<S> a) {
    using T = typename Storage<S>::T;
    const Geom &g = a.g;
    const int count = *a.count;
    const int item = logical_item(count, 4);
    if (item < 0) return;
    const int cell = a.list[item];
    const int lane = threadIdx.x & 63;
    const Nbr nb = neighbours(cell, g);
    const T dv = (T)g.dv, vmax = (T)g.vmax;
    const T idx = (T)(1.0 / g.dx), idy = (T)(1.0 / g.dy);
    const double te = g.tau / a.eps[cell];
    const T dt = (T)g.dt;

    GaussEval<T> ge[2];
    for (int q = 0; q < a.nq; ++q) ge[q].load(a.pq[q] + (size_t)cell * GP_N);

    T fs[C][4];
    T vx0[C], vyc[C];
    Comp<T> s0, sx, sy;
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const int k0 = chunk_node(lane, m);
        const int ia = k0 % g.nv, ib = k0 / g.nv;
        vx0[m] = -vmax + ((T)ia + (T)0.5) * dv;
        vyc[m] = -vmax + ((T)ib + (T)0.5) * dv;
#pragma unroll
        for (int e = 0; e < 4; ++e) fs[m][e] = 0;
        if (k0 < g.nv2) {
            T vx[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) vx[e] = vx0[m] + (T)e * dv;
            T base[4], accL[4] = {0, 0, 0, 0}, accS[4] = {0, 0, 0, 0};
            Storage<S>::load4(a.fn, nb.c + k0, base);
            for (int l = 0; l < a.nl; ++l) {
                T L[4];
                transport4<S>(a.fl[l], nb, k0, vx, vyc[m], idx, idy, g.recon, L);
                const T cl = (T)a.cl[l];
#pragma unroll
                for (int e = 0; e < 4; ++e) accL[e] += cl * L[e];
            }
            for (int q = 0; q < a.nq; ++q) {
                T fj[4];
                Storage<S>::load4(a.fq[q], nb.c + k0, fj);
                const T cq = (T)a.cq[q];
#pragma unroll
                for (int e = 0; e < 4; ++e) accS[e] += cq * (ge[q].hat(vx[e], vyc[m]) - fj[e]);
            }
            const T dtte = (T)(g.dt * te);
#pragma unroll
            for (int e = 0; e < 4; ++e) fs[m][e] = base[e] - dt * accL[e] + dtte * accS[e];
            T c0 = (fs[m][0] + fs[m][1]) + (fs[m][2] + fs[m][3]);
            T cx = (vx[0] * fs[m][0] + vx[1] * fs[m][1]) + (vx[2] * fs[m][2] + vx[3] * fs[m][3]);
            s0.add(c0);
            sx.add(cx);
            sy.add(vyc[m] * c0);
        }
    }
    // ---- first moments (compensated in the arithmetic type)
    const double w = g.w;
    const double rho = w * wave_sum_comp(s0);
    const double ux = w * wave_sum_comp(sx) / rho;
    const double uy = w * wave_sum_comp(sy) / rho;
    // ---- centred second moments
    Comp<T> pxx, pxy, pyy;
    {
        const T uxt = (T)ux, uyt = (T)uy;
#pragma unroll
        for (int m = 0; m < C; ++m) {
            if (chunk_node(lane, m) < g.nv2) {
                T ey = vyc[m] - uyt;
                T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    T ex = vx0[m] + (T)e * dv - uxt;
                    a0 += ex * ex * fs[m][e];
                    a1 += ex * fs[m][e];
                    a2 += fs[m][e];
                }
                pxx.add(a0);
                pxy.add(ey * a1);
                pyy.add(ey * ey * a2);
            }
        }
    }
    const double Pxx = w * wave_sum_comp(pxx), Pxy = w * wave_sum_comp(pxy), Pyy = w * wave_sum_comp(pyy);
    const double Tm = (Pxx + Pyy) / (2.0 * rho);
    int errbits = 0;
    if (!(rho > 0.0)) errbits |= ERR_RHO;
    if (!(Tm > 0.0)) errbits |= ERR_T;
    if (rho != rho || Tm != Tm) errbits |= ERR_NAN;

    if (a.aii > 0.0) {
        // ---- FP64 closed form of the implicit relaxation
        const double beta = g.beta;
        const double lam = g.dt * a.aii * te;
        const double k = lam * (1.0 - beta);
        const double thxx = (Pxx / rho + k * Tm) / (1.0 + k);
        const double thxy = (Pxy / rho) / (1.0 + k);
        const double thyy = (Pyy / rho + k * Tm) / (1.0 + k);
        const double txx = (1.0 - beta) * Tm + beta * thxx;
        const double txy = beta * thxy;
        const double tyy = (1.0 - beta) * Tm + beta * thyy;
        double gp[GP_N];
        if (!gauss_params(rho, ux, uy, Tm, txx, txy, tyy, gp)) errbits |= ERR_SPD;
        GaussEval<T> gi;
        gi.load(gp);
        if (g.correction) {
            // 15 discrete moments of the sampled Gaussian
            T acc[15];
#pragma unroll
            for (int q = 0; q < 15; ++q) acc[q] = 0;
#pragma unroll
            for (int m = 0; m < C; ++m) {
                if (chunk_node(lane, m) < g.nv2) {
                    const T b = (vyc[m] - gi.uy) * gi.ist;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const T vx = vx0[m] + (T)e * dv;
                        const T G = gi.tilde(vx, vyc[m]);
                        const T aa = (vx - gi.ux) * gi.ist;
                        const T a2 = aa * aa, b2 = b * b;
                        const T Ga = G * aa, Gb = G * b, Ga2 = G * a2, Gab = Ga * b, Gb2 = G * b2;
                        acc[0] += G;   acc[1] += Ga;  acc[2] += Gb;
                        acc[3] += Ga2; acc[4] += Gab; acc[5] += Gb2;
                        acc[6] += Ga2 * aa; acc[7] += Ga2 * b; acc[8] += Gab * b; acc[9] += Gb2 * b;
                        acc[10] += Ga2 * a2; acc[11] += Ga2 * aa * b; acc[12] += Ga2 * b2;
                        acc[13] += Gab * b2; acc[14] += Gb2 * b2;
                    }
                }
            }
            double Sm[15];
#pragma unroll
            for (int q = 0; q < 15; ++q) Sm[q] = w * wave_sum((double)acc[q]);
            if (!solve_correction(Sm, rho, Tm, txx, txy, tyy, gp)) errbits |= ERR_SPD;
            gi.load(gp);
        }
        // ---- relaxation: the stage's single write
        const T lamt = (T)lam, inv1 = (T)(1.0 / (1.0 + lam));
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const int k0 = chunk_node(lane, m);
            if (k0 < g.nv2) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T vx = vx0[m] + (T)e * dv;
                    fs[m][e] = (fs[m][e] + lamt * gi.hat(vx, vyc[m])) * inv1;
                }
                Storage<S>::store4(a.fout, nb.c + k0, fs[m]);
            }
        }
        if (lane == 0) {
            double *o = a.pout + (size_t)cell * GP_N;
#pragma unroll
            for (int q = 0; q < GP_N; ++q) o[q] = gp[q];
        }
    } else {
        // final combination: fs is f^{n+1}
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const int k0 = chunk_node(lane, m);
            if (k0 < g.nv2) Storage<S>::store4(a.fout, nb.c + k0, fs[m]);
        }
    }
    if (a.emit) {
        // L1 distance to the (uncorrected) sampled Maxwellian of the result's
        // moments; the relaxation keeps rho, u, T of f*, so these are the
        // moments of the written values up to rounding.
        const T l2p = (T)log2(rho / (2.0 * kPi * Tm));
        const T qm = (T)(-0.5 * kLog2e / Tm);
        const T uxt = (T)ux, uyt = (T)uy;
        T l1 = 0;
#pragma unroll
        for (int m = 0; m < C; ++m) {
            if (chunk_node(lane, m) < g.nv2) {
                const T ey = vyc[m] - uyt;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T ex = vx0[m] + (T)e * dv - uxt;
                    const T M = fast_exp2(l2p + qm * (ex * ex + ey * ey));
                    l1 += fabs(fs[m][e] - M);
                }
            }
        }
        const double L1 = w * wave_sum((double)l1);
        if (lane == 0) a.l1out[cell] = L1;
    }
    if (lane == 0) {
        const size_t nc = (size_t)a.nc;
        a.Uout[cell] = rho;
        a.Uout[nc + cell] = rho * ux;
        a.Uout[2 * nc + cell] = rho * uy;
        a.Uout[3 * nc + cell] = 0.5 * rho * (ux * ux + uy * uy) + rho * Tm;
    }
    raise_err(a.err, errbits);
}

// ---------------------------------------------------------------- fills

// f = Mhat(U) at the listed cells (eq. Coupling_FluKin): the corrected sampled
// Maxwellian, i.e. the corrected Gaussian with Tt = T I.
template <class S, int C>
__global__ __launch_bounds__(256) void fill_maxwellian_kernel(FillArgs<S> a) {
    using T = typename Storage<S>::T;
    const Geom &g = a.g;
    const int item = logical_item(*a.count, 4);
    if (item < 0) return;
    const int cell = a.list[item];
    const int lane = threadIdx.x & 63;
    const size_t nc = (size_t)a.nc;
    const double rho = a.U[cell];
    const double ux = a.U[nc + cell] / rho, uy = a.U[2 * nc + cell] / rho;
    const double Tm = (a.U[3 * nc + cell] - 0.5 * rho * (ux * ux + uy * uy)) / rho;
    int errbits = 0;
    double gp[GP_N];
    if (!gauss_params(rho, ux, uy, Tm, Tm, 0.0, Tm, gp)) errbits |= ERR_SPD;
    GaussEval<T> gi;
    gi.load(gp);
    const T dv = (T)g.dv, vmax = (T)g.vmax;
    if (g.correction) {
        T acc[15];
#pragma unroll
        for (int q = 0; q < 15; ++q) acc[q] = 0;
#pragma unroll
        for (int m = 0; m < C; ++m) {
            const int k0 = chunk_node(lane, m);
            if (k0 < g.nv2) {
                const T vy = -vmax + ((T)(k0 / g.nv) + (T)0.5) * dv;
                const T vx0 = -vmax + ((T)(k0 % g.nv) + (T)0.5) * dv;
                const T b = (vy - gi.uy) * gi.ist;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const T vx = vx0 + (T)e * dv;
                    const T G = gi.tilde(vx, vy);
                    const T aa = (vx - gi.ux) * gi.ist;
                    const T a2 = aa * aa, b2 = b * b;
                    const T Ga = G * aa, Gb = G * b, Ga2 = G * a2, Gab = Ga * b, Gb2 = G * b2;
                    acc[0] += G;   acc[1] += Ga;  acc[2] += Gb;
                    acc[3] += Ga2; acc[4] += Gab; acc[5] += Gb2;
                    acc[6] += Ga2 * aa; acc[7] += Ga2 * b; acc[8] += Gab * b; acc[9] += Gb2 * b;
                    acc[10] += Ga2 * a2; acc[11] += Ga2 * aa * b; acc[12] += Ga2 * b2;
                    acc[13] += Gab * b2; acc[14] += Gb2 * b2;
                }
            }
        }
        double Sm[15];
#pragma unroll
        for (int q = 0; q < 15; ++q) Sm[q] = g.w * wave_sum((double)acc[q]);
        if (!solve_correction(Sm, rho, Tm, Tm, 0.0, Tm, gp)) errbits |= ERR_SPD;
        gi.load(gp);
    }
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const int k0 = chunk_node(lane, m);
        if (k0 < g.nv2) {
            const T vy = -vmax + ((T)(k0 / g.nv) + (T)0.5) * dv;
            const T vx0 = -vmax + ((T)(k0 % g.nv) + (T)0.5) * dv;
            T v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) v[e] = gi.hat(vx0 + (T)e * dv, vy);
            Storage<S>::store4(a.f, (size_t)cell * g.nv2 + k0, v);
        }
    }
    raise_err(a.err, errbits);
}

// U = moments(f) and the L1 distance at the listed cells (eq. Coupling_KinFlu,
// eq. eqKintoFluid1).
template <class S, int C>
__global__ __launch_bounds__(256) void moments_kernel(MomArgs<S> a) {
    using T = typename Storage<S>::T;
    const Geom &g = a.g;
    const int item = logical_item(*a.count, 4);
    if (item < 0) return;
    const int cell = a.list[item];
    const int lane = threadIdx.x & 63;
    const T dv = (T)g.dv, vmax = (T)g.vmax;
    T fv[C][4];
    T vx0[C], vyc[C];
    Comp<T> s0, sx, sy;
#pragma unroll
    for (int m = 0; m < C; ++m) {
        const int k0 = chunk_node(lane, m);
        vx0[m] = -vmax + ((T)(k0 % g.nv) + (T)0.5) * dv;
        vyc[m] = -vmax + ((T)(k0 / g.nv) + (T)0.5) * dv;
#pragma unroll
        for (int e = 0; e < 4; ++e) fv[m][e] = 0;
        if (k0 < g.nv2) {
            Storage<S>::load4(a.f, (size_t)cell * g.nv2 + k0, fv[m]);
            T c0 = (fv[m][0] + fv[m][1]) + (fv[m][2] + fv[m][3]);
            T cx = (vx0[m] * fv[m][0] + (vx0[m] + dv) * fv[m][1]) +
                   ((vx0[m] + (T)2 * dv) * fv[m][2] + (vx0[m] + (T)3 * dv) * fv[m][3]);
            s0.add(c0);
            sx.add(cx);
            sy.add(vyc[m] * c0);
        }
    }
    const double w = g.w;
    const double rho = w * wave_sum_comp(s0);
    const double ux = w * wave_sum_comp(sx) / rho;
    const double uy = w * wave_sum_comp(sy) / rho;
    Comp<T> pt;
    const T uxt = (T)ux, uyt = (T)uy;
#pragma unroll
    for (int m = 0; m < C; ++m) {
        if (chunk_node(lane, m) < g.nv2) {
            T ey = vyc[m] - uyt, acc = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                T ex = vx0[m] + (T)e * dv - uxt;
                acc += (ex * ex + ey * ey) * fv[m][e];
            }
            pt.add(acc);
        }
    }
    const double Tm = w * wave_sum_comp(pt) / (2.0 * rho);
    const T l2p = (T)log2(rho / (2.0 * kPi * Tm));
    const T qm = (T)(-0.5 * kLog2e / Tm);
    T l1 = 0;
#pragma unroll
    for (int m = 0; m < C; ++m) {
        if (chunk_node(lane, m) < g.nv2) {
            T ey = vyc[m] - uyt;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                T ex = vx0[m] + (T)e * dv - uxt;
                l1 += fabs(fv[m][e] - fast_exp2(l2p + qm * (ex * ex + ey * ey)));
            }
        }
    }
    const double L1 = w * wave_sum((double)l1);
    int errbits = 0;
    if (!(rho > 0.0)) errbits |= ERR_RHO;
    if (!(Tm > 0.0)) errbits |= ERR_T;
    if (lane == 0) {
        const size_t nc = (size_t)a.nc;
        a.U[cell] = rho;
        a.U[nc + cell] = rho * ux;
        a.U[2 * nc + cell] = rho * uy;
        a.U[3 * nc + cell] = 0.5 * rho * (ux * ux + uy * uy) + rho * Tm;
        if (a.l1) a.l1[cell] = L1;
    }
    raise_err(a.err, errbits);
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

static inline int chunks_for(int nv2) {
    int need = (nv2 + 255) / 256;
    if (need <= 1) return 1;
    if (need <= 2) return 2;
    if (need <= 4) return 4;
    if (need <= 9) return 9;
    return 16;
}

static inline unsigned grid_for(int nmax) {
    int nblk = (nmax + 3) / 4;
    int per = (nblk + 7) / 8;
    return (unsigned)(per * 8 > 0 ? per * 8 : 8);
}

template <class S, int C> static void stage_c(const StageArgs<S> &a, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((stage_kernel<S, C>), dim3(grid), dim3(256), 0, st, a);
}
template <class S, int C> static void fill_c(const FillArgs<S> &a, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((fill_maxwellian_kernel<S, C>), dim3(grid), dim3(256), 0, st, a);
}
template <class S, int C> static void moments_c(const MomArgs<S> &a, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((moments_kernel<S, C>), dim3(grid), dim3(256), 0, st, a);
}

#define ESBGK_DISPATCH_C(FN, S, A, GRID, ST)          \
    switch (chunks_for((A).g.nv2)) {                  \
        case 1: FN<S, 1>(A, GRID, ST); break;          \
        case 2: FN<S, 2>(A, GRID, ST); break;          \
        case 4: FN<S, 4>(A, GRID, ST); break;          \
        case 9: FN<S, 9>(A, GRID, ST); break;          \
        default: FN<S, 16>(A, GRID, ST); break;        \
    }

template <class S>
hipError_t launch_stage(const StageArgs<S> &a, int nmax, hipStream_t st) {
    ESBGK_DISPATCH_C(stage_c, S, a, grid_for(nmax), st);
    return hipGetLastError();
}

template <class S>
hipError_t launch_fill(const FillArgs<S> &a, int nmax, hipStream_t st) {
    ESBGK_DISPATCH_C(fill_c, S, a, grid_for(nmax), st);
    return hipGetLastError();
}

template <class S>
hipError_t launch_moments(const MomArgs<S> &a, int nmax, hipStream_t st) {
    ESBGK_DISPATCH_C(moments_c, S, a, grid_for(nmax), st);
    return hipGetLastError();
}

template <class S>
hipError_t launch_from_f64(const double *in, void *out, size_t n, hipStream_t st) {
    size_t n4 = n / 4;
    unsigned grid = (unsigned)((n4 + 255) / 256 < 65536 ? (n4 + 255) / 256 : 65536);
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL((f_from_f64_kernel<S>), dim3(grid), dim3(256), 0, st, in, (S *)out, n4);
    return hipGetLastError();
}

template <class S>
hipError_t launch_to_f64(const void *in, double *out, size_t n, hipStream_t st) {
    size_t n4 = n / 4;
    unsigned grid = (unsigned)((n4 + 255) / 256 < 65536 ? (n4 + 255) / 256 : 65536);
    if (grid == 0) grid = 1;
    hipLaunchKernelGGL((f_to_f64_kernel<S>), dim3(grid), dim3(256), 0, st, (const S *)in, out, n4);
    return hipGetLastError();
}

#define ESBGK_INST(S)                                                                        \
    template hipError_t launch_stage<S>(const StageArgs<S> &, int, hipStream_t);             \
    template hipError_t launch_fill<S>(const FillArgs<S> &, int, hipStream_t);               \
    template hipError_t launch_moments<S>(const MomArgs<S> &, int, hipStream_t);             \
    template hipError_t launch_from_f64<S>(const double *, void *, size_t, hipStream_t);     \
    template hipError_t launch_to_f64<S>(const void *, double *, size_t, hipStream_t);

ESBGK_INST(double)
ESBGK_INST(float)
ESBGK_INST(bf16_t)

}  // namespace esbgk
