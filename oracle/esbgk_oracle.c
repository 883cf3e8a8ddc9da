/*
 * esbgk_oracle.c -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.
 *
 * A plain, slow, FP64 CPU reference ("oracle") for the coupled IMEX
 * domain-decomposition ES-BGK scheme of Caparello & Tenna, "A Coupled IMEX
 * Domain Decomposition Method for High-Order Time Integration of the ES-BGK
 * Model of the Boltzmann Equation" (arXiv 2512.03586).  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load this library;
 * the GPU path shares no code with it.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math), so
 * every + - * / sqrt is a correctly rounded IEEE double operation executed in
 * source order.
 *
 * Each function names the passage of the paper it follows.  Where the paper is
 * silent the function states the reading it takes; the list of readings is
 * repeated in the project's design notes.
 *
 * Conventions (Sec. 3.2, "Velocity and Spatial Discretization"):
 *   cells i = 0..nx-1, j = 0..ny-1 on [0,lx] x [0,ly], cell index c = i + nx*j;
 *   velocity nodes a, b = 0..nv-1 per direction (nv counts nodes per direction),
 *   midpoint nodes v = -V + (a + 1/2) dv with dv = 2V/nv  (reading: the paper
 *   only fixes a square grid of step dv), quadrature weight w = dv^2;
 *   node index k = a + nv*b (x-velocity fastest); f[c*nv*nv + k].
 * Conserved variables U (SoA, 4 planes of nc): rho, rho*ux, rho*uy, E with
 *   E = rho|u|^2/2 + rho*T (d_v = 2, so gamma = 2 and P = rho*T; Sec. 2).
 *
 * Parity: every function here is pinned by the tests in tests/test_oracle_*.py
 * against closed forms, invariants, special cases or brute force.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nv;
    int32_t scheme;      /* 0 = ARS(2,2,2), 1 = ARS(2,3,3) */
    int32_t recon;       /* 0 = first-order upwind, 1 = minmod (2nd order) */
    int32_t correction;  /* 0 = none (sampled Gaussian), 1 = six-moment correction */
    int32_t ce_set;      /* 0 = paper's Chapman-Enskog constants, 1 = 2D-consistent */
    int32_t coupling;    /* 0 = at every stage (Algorithm 1), 1 = once per step (LOC) */
    double lx, ly, vmax;
    double beta, tau, dt;
    double eta, delta;
} orc_cfg;

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ grids */

static double orc_dv(const orc_cfg *c) { return 2.0 * c->vmax / (double)c->nv; }

/* Velocity of node k (Sec. 3.2; midpoint-node reading). */
static void orc_vel(const orc_cfg *c, int k, double *vx, double *vy)
{
    double dv = orc_dv(c);
    int a = k % c->nv, b = k / c->nv;
    *vx = -c->vmax + ((double)a + 0.5) * dv;
    *vy = -c->vmax + ((double)b + 0.5) * dv;
}

void orc_velocity_nodes(const orc_cfg *c, double *vx, double *vy)
{
    int nv2 = c->nv * c->nv;
    for (int k = 0; k < nv2; ++k) orc_vel(c, k, &vx[k], &vy[k]);
}

/* ------------------------------------------------------------ tableaux */

/* IMEX Runge-Kutta tableaux, 3 stages, row-major 3x3.
 * ARS(2,3,3): the two tableaux printed in Sec. 3.4.2, alpha = (3+sqrt 3)/6.
 * ARS(2,2,2): reading for the unnamed "second-order IMEX" scheme; the
 * second-order member of the same Ascher-Ruuth-Spiteri family the paper cites,
 * gamma = 1 - 1/sqrt 2, delta = 1 - 1/(2 gamma).  Explicit (At, bt), implicit (A, b). */
void orc_tableau(int scheme, double *At, double *bt, double *A, double *b)
{
    memset(At, 0, 9 * sizeof(double));
    memset(A, 0, 9 * sizeof(double));
    if (scheme == 1) {
        double al = (3.0 + sqrt(3.0)) / 6.0;
        At[3] = al;
        At[6] = al - 1.0; At[7] = 2.0 - 2.0 * al;
        bt[0] = 0.0; bt[1] = 0.5; bt[2] = 0.5;
        A[4] = al;
        A[7] = 1.0 - 2.0 * al; A[8] = al;
        b[0] = 0.0; b[1] = 0.5; b[2] = 0.5;
    } else {
        double g = 1.0 - 1.0 / sqrt(2.0);
        double d = 1.0 - 1.0 / (2.0 * g);
        At[3] = g;
        At[6] = d; At[7] = 1.0 - d;
        bt[0] = d; bt[1] = 1.0 - d; bt[2] = 0.0;
        A[4] = g;
        A[7] = 1.0 - g; A[8] = g;
        b[0] = 0.0; b[1] = 1.0 - g; b[2] = g;
    }
}

/* -------------------------------------------------------------- moments */

/* Density, mean velocity, temperature and the tensor Theta of one cell's
 * distribution (hypothesis H3 and the definition of Theta in Sec. 2):
 *   rho = int f, u = int v f / rho, Theta = int (v-u)(v-u) f / rho,
 *   T = trace(Theta)/d_v with d_v = 2.  Two passes (centred second moments).
 * out = {rho, ux, uy, T, Thxx, Thxy, Thyy}. */
void orc_moments(const orc_cfg *c, const double *fc, double *out)
{
    int nv2 = c->nv * c->nv;
    double w = orc_dv(c) * orc_dv(c);
    double s0 = 0, sx = 0, sy = 0;
    for (int k = 0; k < nv2; ++k) {
        double vx, vy;
        orc_vel(c, k, &vx, &vy);
        s0 += fc[k];
        sx += vx * fc[k];
        sy += vy * fc[k];
    }
    double rho = w * s0;
    double ux = w * sx / rho, uy = w * sy / rho;
    double pxx = 0, pxy = 0, pyy = 0;
    for (int k = 0; k < nv2; ++k) {
        double vx, vy;
        orc_vel(c, k, &vx, &vy);
        double ex = vx - ux, ey = vy - uy;
        pxx += ex * ex * fc[k];
        pxy += ex * ey * fc[k];
        pyy += ey * ey * fc[k];
    }
    pxx *= w; pxy *= w; pyy *= w;
    out[0] = rho;
    out[1] = ux;
    out[2] = uy;
    out[3] = (pxx + pyy) / (2.0 * rho);
    out[4] = pxx / rho;
    out[5] = pxy / rho;
    out[6] = pyy / rho;
}

/* ------------------------------------------------- Maxwellian, Gaussian */

/* Sampled Maxwellian M = rho/(2 pi T) exp(-|v-u|^2/(2T)) (H3 with d_v = 2). */
void orc_maxwellian(const orc_cfg *c, double rho, double ux, double uy, double T, double *m)
{
    int nv2 = c->nv * c->nv;
    double pref = rho / (2.0 * ORC_PI * T);
    for (int k = 0; k < nv2; ++k) {
        double vx, vy;
        orc_vel(c, k, &vx, &vy);
        double ex = vx - ux, ey = vy - uy;
        m[k] = pref * exp(-(ex * ex + ey * ey) / (2.0 * T));
    }
}

/* Sampled anisotropic Gaussian of Sec. 2:
 *   G = rho / sqrt(det(2 pi Tt)) exp(-(v-u)^T Tt^{-1} (v-u) / 2),
 * for a symmetric positive-definite 2x2 tensor Tt = [[txx, txy], [txy, tyy]];
 * in 2D sqrt(det(2 pi Tt)) = 2 pi sqrt(det Tt).  Returns -1 if Tt is not
 * positive definite. */
int orc_gaussian_tilde(const orc_cfg *c, double rho, double ux, double uy,
                       double txx, double txy, double tyy, double *g)
{
    int nv2 = c->nv * c->nv;
    double det = txx * tyy - txy * txy;
    if (!(det > 0.0) || !(txx > 0.0)) return -1;
    double ixx = tyy / det, ixy = -txy / det, iyy = txx / det;
    double pref = rho / (2.0 * ORC_PI * sqrt(det));
    for (int k = 0; k < nv2; ++k) {
        double vx, vy;
        orc_vel(c, k, &vx, &vy);
        double ex = vx - ux, ey = vy - uy;
        double q = ixx * ex * ex + 2.0 * ixy * ex * ey + iyy * ey * ey;
        g[k] = pref * exp(-0.5 * q);
    }
    return 0;
}

/* Solve the n x n system M x = r by Gaussian elimination with partial
 * pivoting (M and r are overwritten).  Returns -1 if singular. */
static int orc_solve(int n, double *M, double *r, double *x)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = fabs(M[col * n + col]);
        for (int row = col + 1; row < n; ++row) {
            double v = fabs(M[row * n + col]);
            if (v > best) { best = v; piv = row; }
        }
        if (!(best > 0.0)) return -1;
        if (piv != col) {
            for (int k = 0; k < n; ++k) {
                double t = M[col * n + k]; M[col * n + k] = M[piv * n + k]; M[piv * n + k] = t;
            }
            double t = r[col]; r[col] = r[piv]; r[piv] = t;
        }
        for (int row = col + 1; row < n; ++row) {
            double fac = M[row * n + col] / M[col * n + col];
            for (int k = col; k < n; ++k) M[row * n + k] -= fac * M[col * n + k];
            r[row] -= fac * r[col];
        }
    }
    for (int row = n - 1; row >= 0; --row) {
        double s = r[row];
        for (int k = row + 1; k < n; ++k) s -= M[row * n + k] * x[k];
        x[row] = s / M[row * n + row];
    }
    return 0;
}

/* Discrete-conservation correction of the sampled Gaussian (a reading: the
 * paper states that the scheme conserves mass, momentum and energy, Sec. 3.6,
 * but does not say how the sampled Gaussian is made to carry the right
 * discrete moments).  With xi = (v-u)/sqrt(T) and
 * psi = (1, xi_x, xi_y, xi_x^2, xi_x xi_y, xi_y^2), find c such that
 * Ghat = Gtilde * (c . psi) has discrete moments w*sum Ghat psi_m equal to the
 * continuous ones, (rho, 0, 0, rho txx/T, rho txy/T, rho tyy/T):
 * A c = t with the Gram matrix A_mn = w sum Gtilde psi_m psi_n.
 * coef (may be NULL) receives c. */
int orc_gaussian_hat(const orc_cfg *c, double rho, double ux, double uy, double T,
                     double txx, double txy, double tyy, double *g, double *coef)
{
    if (orc_gaussian_tilde(c, rho, ux, uy, txx, txy, tyy, g) != 0) return -1;
    double cc[6] = {1, 0, 0, 0, 0, 0};
    if (c->correction) {
        int nv2 = c->nv * c->nv;
        double w = orc_dv(c) * orc_dv(c);
        double sq = sqrt(T);
        double M[36];
        memset(M, 0, sizeof M);
        for (int k = 0; k < nv2; ++k) {
            double vx, vy;
            orc_vel(c, k, &vx, &vy);
            double a = (vx - ux) / sq, b = (vy - uy) / sq;
            double psi[6] = {1.0, a, b, a * a, a * b, b * b};
            for (int m = 0; m < 6; ++m)
                for (int n = 0; n < 6; ++n) M[m * 6 + n] += g[k] * psi[m] * psi[n];
        }
        for (int m = 0; m < 36; ++m) M[m] *= w;
        double r[6] = {rho, 0.0, 0.0, rho * txx / T, rho * txy / T, rho * tyy / T};
        if (orc_solve(6, M, r, cc) != 0) return -2;
        for (int k = 0; k < nv2; ++k) {
            double vx, vy;
            orc_vel(c, k, &vx, &vy);
            double a = (vx - ux) / sq, b = (vy - uy) / sq;
            g[k] *= cc[0] + cc[1] * a + cc[2] * b + cc[3] * a * a + cc[4] * a * b + cc[5] * b * b;
        }
    }
    if (coef) memcpy(coef, cc, sizeof cc);
    return 0;
}

/* Maxwellian with the same correction: Ghat with Tt = T I (Sec. 2: for
 * Theta = T I the tensor Tt reduces to T I and G to M).  This is the
 * distribution a fluid cell supplies (eq. Coupling_FluKin). */
int orc_maxwellian_hat(const orc_cfg *c, double rho, double ux, double uy, double T, double *m)
{
    return orc_gaussian_hat(c, rho, ux, uy, T, T, 0.0, T, m, NULL);
}

/* ES tensor Tt = (1-beta) T I + beta Theta (Sec. 2). */
static void orc_es_tensor(double beta, double T, double thxx, double thxy, double thyy,
                          double *txx, double *txy, double *tyy)
{
    *txx = (1.0 - beta) * T + beta * thxx;
    *txy = beta * thxy;
    *tyy = (1.0 - beta) * T + beta * thyy;
}

/* G[f] for one cell: moments of f, ES tensor, corrected Gaussian. */
int orc_gaussian_of(const orc_cfg *c, const double *fc, double *g)
{
    double mo[7], txx, txy, tyy;
    orc_moments(c, fc, mo);
    orc_es_tensor(c->beta, mo[3], mo[4], mo[5], mo[6], &txx, &txy, &tyy);
    return orc_gaussian_hat(c, mo[0], mo[1], mo[2], mo[3], txx, txy, tyy, g, NULL);
}

/* ---------------------------------------------------------- relaxation */

/* Implicit relaxation of one IMEX stage for one cell (eq. RKEI1 with the ES-BGK
 * source (tau/eps)(G[f] - f) taken implicitly, the relaxation rate read as a
 * single tau/eps):  f = fstar + lam (G[f] - f),  lam = dt a_ii tau/eps.
 * Taking the discrete moments of this equation (the corrected G carries exact
 * discrete moments, H1) gives rho, u, T of f equal to those of fstar and
 *   Theta = (Theta* + lam (1-beta) T I) / (1 + lam (1-beta)),
 * so G[f] is known before f and f = (fstar + lam G) / (1 + lam).
 * ghat (may be NULL) receives G[f]; mo (may be NULL) receives
 * {rho, ux, uy, T, txx, txy, tyy}. */
int orc_relax_cell(const orc_cfg *c, const double *fstar, double lam, double *fout,
                   double *ghat, double *mo_out)
{
    int nv2 = c->nv * c->nv;
    double mo[7];
    orc_moments(c, fstar, mo);
    double rho = mo[0], ux = mo[1], uy = mo[2], T = mo[3];
    double k = lam * (1.0 - c->beta);
    double thxx = (mo[4] + k * T) / (1.0 + k);
    double thxy = mo[5] / (1.0 + k);
    double thyy = (mo[6] + k * T) / (1.0 + k);
    double txx, txy, tyy;
    orc_es_tensor(c->beta, T, thxx, thxy, thyy, &txx, &txy, &tyy);
    double *g = ghat ? ghat : (double *)malloc(nv2 * sizeof(double));
    int rc = orc_gaussian_hat(c, rho, ux, uy, T, txx, txy, tyy, g, NULL);
    if (rc == 0)
        for (int kk = 0; kk < nv2; ++kk) fout[kk] = (fstar[kk] + lam * g[kk]) / (1.0 + lam);
    if (mo_out) {
        mo_out[0] = rho; mo_out[1] = ux; mo_out[2] = uy; mo_out[3] = T;
        mo_out[4] = txx; mo_out[5] = txy; mo_out[6] = tyy;
    }
    if (!ghat) free(g);
    return rc;
}

/* ----------------------------------------------------------- transport */

/* minmod(a, b) = 0 when a and b differ in sign or one is zero, otherwise the
 * argument of smaller magnitude.  The sign test is done on the signs (not on
 * the product a*b, which underflows to zero for tiny tail values). */
static double orc_minmod(double a, double b)
{
    if (!((a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0))) return 0.0;
    return a > 0.0 ? fmin(a, b) : fmax(a, b);
}

static int orc_wrap(int i, int n) { return ((i % n) + n) % n; }

/* Face flux of one direction at the face between cells p (left) and q (right)
 * for velocity component s: upwind flux s^+ f^- + s^- f^+ on face values of a
 * piecewise-constant (recon 0) or minmod-limited piecewise-linear (recon 1)
 * reconstruction.  fm2..fp1 are the values in cells p-1, p, q, q+1.  This is
 * the Lax-Friedrichs flux of Sec. 3.2 with dissipation |s|, applied to the
 * reconstruction the workloads ask for (upwind / second-order limited). */
static double orc_face_flux(int recon, double s, double fpm, double fp, double fq, double fqp)
{
    double sp = 0.0, sq = 0.0;
    if (recon == 1) {
        sp = orc_minmod(fp - fpm, fq - fp);
        sq = orc_minmod(fq - fp, fqp - fq);
    }
    double fl = fp + 0.5 * sp;   /* left state at the face  */
    double fr = fq - 0.5 * sq;   /* right state at the face */
    return fmax(s, 0.0) * fl + fmin(s, 0.0) * fr;
}

/* Finite-volume transport operator L(f) ~ v . grad_x f at one cell and one
 * node (semidiscrete ES-BGK system, Sec. 3.4), periodic boundaries
 * (reading for the periodic workloads):
 *   L = (F_{i+1/2} - F_{i-1/2}) / dx + (G_{j+1/2} - G_{j-1/2}) / dy. */
static double orc_transport_node(const orc_cfg *c, const double *f, int i, int j, int k,
                                 double vx, double vy)
{
    int nx = c->nx, ny = c->ny, nv2 = c->nv * c->nv;
    double dx = c->lx / nx, dy = c->ly / ny;
#define F(ii, jj) f[((size_t)orc_wrap(jj, ny) * nx + orc_wrap(ii, nx)) * nv2 + k]
    double fxp = orc_face_flux(c->recon, vx, F(i - 1, j), F(i, j), F(i + 1, j), F(i + 2, j));
    double fxm = orc_face_flux(c->recon, vx, F(i - 2, j), F(i - 1, j), F(i, j), F(i + 1, j));
    double fyp = orc_face_flux(c->recon, vy, F(i, j - 1), F(i, j), F(i, j + 1), F(i, j + 2));
    double fym = orc_face_flux(c->recon, vy, F(i, j - 2), F(i, j - 1), F(i, j), F(i, j + 1));
#undef F
    return (fxp - fxm) / dx + (fyp - fym) / dy;
}

/* L(f) on every cell and node.  f and out are full nc*nv2 arrays. */
void orc_transport(const orc_cfg *c, const double *f, double *out)
{
    int nx = c->nx, ny = c->ny, nv2 = c->nv * c->nv;
#pragma omp parallel for schedule(static)
    for (int cell = 0; cell < nx * ny; ++cell) {
        int i = cell % nx, j = cell / nx;
        for (int k = 0; k < nv2; ++k) {
            double vx, vy;
            orc_vel(c, k, &vx, &vy);
            out[(size_t)cell * nv2 + k] = orc_transport_node(c, f, i, j, k, vx, vy);
        }
    }
}

/* --------------------------------------------------------------- Euler */

/* Physical Euler flux in direction d (0 = x, 1 = y) of U = (rho, mx, my, E),
 * eq. Euler_Compact with P = (gamma-1)(E - rho|u|^2/2), gamma = 2. */
void orc_euler_flux(const double *U, int d, double *F)
{
    double rho = U[0], ux = U[1] / rho, uy = U[2] / rho, E = U[3];
    double P = (E - 0.5 * rho * (ux * ux + uy * uy));
    double un = d == 0 ? ux : uy;
    F[0] = rho * un;
    F[1] = U[1] * un + (d == 0 ? P : 0.0);
    F[2] = U[2] * un + (d == 1 ? P : 0.0);
    F[3] = un * (E + P);
}

/* Rusanov (local Lax-Friedrichs) numerical flux between face states UL, UR,
 * with speed max(|u_n| + sqrt(gamma P / rho)) over both states (reading of
 * the Lax-Friedrichs flux of Sec. 3.2; gamma = 2). */
void orc_rusanov(const double *UL, const double *UR, int d, double *Fh)
{
    double FL[4], FR[4];
    orc_euler_flux(UL, d, FL);
    orc_euler_flux(UR, d, FR);
    double aL, aR;
    {
        double rho = UL[0], ux = UL[1] / rho, uy = UL[2] / rho;
        double P = UL[3] - 0.5 * rho * (ux * ux + uy * uy);
        aL = fabs(d == 0 ? ux : uy) + sqrt(2.0 * P / rho);
    }
    {
        double rho = UR[0], ux = UR[1] / rho, uy = UR[2] / rho;
        double P = UR[3] - 0.5 * rho * (ux * ux + uy * uy);
        aR = fabs(d == 0 ? ux : uy) + sqrt(2.0 * P / rho);
    }
    double a = fmax(aL, aR);
    for (int q = 0; q < 4; ++q) Fh[q] = 0.5 * (FL[q] + FR[q]) - 0.5 * a * (UR[q] - UL[q]);
}

/* Face flux between cells p and q in direction d, with the same reconstruction
 * as the kinetic transport applied component-wise to conserved variables. */
static void orc_euler_face(const orc_cfg *c, const double *U, size_t nc, size_t cpm, size_t cp,
                           size_t cq, size_t cqp, int d, double *Fh)
{
    double UL[4], UR[4];
    for (int q = 0; q < 4; ++q) {
        double a = U[q * nc + cpm], b = U[q * nc + cp], e = U[q * nc + cq], g = U[q * nc + cqp];
        double sp = 0.0, sq = 0.0;
        if (c->recon == 1) {
            sp = orc_minmod(b - a, e - b);
            sq = orc_minmod(e - b, g - e);
        }
        UL[q] = b + 0.5 * sp;
        UR[q] = e - 0.5 * sq;
    }
    orc_rusanov(UL, UR, d, Fh);
}

/* Semidiscrete Euler divergence Phi(U) (eq. semidiscrete_Euler) at every cell,
 * periodic.  U and Phi are SoA [4][nc]. */
void orc_euler_phi(const orc_cfg *c, const double *U, double *Phi)
{
    int nx = c->nx, ny = c->ny;
    size_t nc = (size_t)nx * ny;
    double dx = c->lx / nx, dy = c->ly / ny;
#define CI(ii, jj) ((size_t)orc_wrap(jj, ny) * nx + orc_wrap(ii, nx))
#pragma omp parallel for schedule(static)
    for (int cell = 0; cell < nx * ny; ++cell) {
        int i = cell % nx, j = cell / nx;
        double Fp[4], Fm[4], Gp[4], Gm[4];
        orc_euler_face(c, U, nc, CI(i - 1, j), CI(i, j), CI(i + 1, j), CI(i + 2, j), 0, Fp);
        orc_euler_face(c, U, nc, CI(i - 2, j), CI(i - 1, j), CI(i, j), CI(i + 1, j), 0, Fm);
        orc_euler_face(c, U, nc, CI(i, j - 1), CI(i, j), CI(i, j + 1), CI(i, j + 2), 1, Gp);
        orc_euler_face(c, U, nc, CI(i, j - 2), CI(i, j - 1), CI(i, j), CI(i, j + 1), 1, Gm);
        for (int q = 0; q < 4; ++q) Phi[q * nc + cell] = (Fp[q] - Fm[q]) / dx + (Gp[q] - Gm[q]) / dy;
    }
#undef CI
}

/* ----------------------------------------------------------- indicator */

/* L1_v distance between a cell's distribution and the (uncorrected, sampled)
 * Maxwellian with the same moments, left-hand side of eq. eqKintoFluid1. */
double orc_l1_to_maxwellian(const orc_cfg *c, const double *fc)
{
    int nv2 = c->nv * c->nv;
    double w = orc_dv(c) * orc_dv(c);
    double mo[7];
    orc_moments(c, fc, mo);
    double *m = (double *)malloc(nv2 * sizeof(double));
    orc_maxwellian(c, mo[0], mo[1], mo[2], mo[3], m);
    double s = 0.0;
    for (int k = 0; k < nv2; ++k) s += fabs(fc[k] - m[k]);
    free(m);
    return w * s;
}

/* Regime indicator of Sec. 3.1.2 for every cell.
 * prim is SoA [4][nc] = (rho, ux, uy, T); eps the local Knudsen number;
 * l1 the L1 distance of eq. eqKintoFluid1 (read only for cells with
 * mask_old = 1); mask 1 = kinetic.
 *   A = S_1 - I = -(eps/(tau(1-beta))) D(u) - cS (ck eps/(tau sqrt T))^2 gradT gradT^T
 * with mu/(rho T) = 1/(tau(1-beta)) and kappa/(rho T^{3/2}) = ck/(tau sqrt T),
 * D(u) = grad u + grad u^T - cD div(u) I (the identity dropped in the printed
 * definition is restored).  Paper constants (ce_set 0): cD = 2/3, ck = 5/2,
 * cS = 2/3 (derived there for d_v = 3); 2D-consistent set (ce_set 1): 1, 2, 1.
 * Gradients are central differences (reading).  The largest |eigenvalue| of
 * the symmetric 2x2 matrix A is |m| + sqrt(h^2 + A12^2), m = (A11+A22)/2,
 * h = (A11-A22)/2.  Fluid -> kinetic when it exceeds eta (criterion
 * crit:CompEuler); kinetic -> fluid only when it does not and the L1 distance
 * is <= delta (Remark and eq. eqKintoFluid1):
 *   mask_new = crit_S || (mask_old && l1 > delta).
 * The decision is evaluated without square roots, through the exact
 * equivalences (ck eps/(tau sqrt T))^2 = (ck eps)^2/(tau^2 T) and
 * |m| + sqrt(q) > eta <=> (eta - |m| < 0 or q > (eta - |m|)^2): it is then a
 * composition of correctly rounded + - * / only.  The operation order below is
 * part of the contract with the GPU indicator; the returned lambda (a report,
 * not used in the decision) takes one square root. */
void orc_indicator(const orc_cfg *c, const double *prim, const double *eps, const double *l1,
                   const uint8_t *mask_old, uint8_t *mask_new, double *lam_out)
{
    int nx = c->nx, ny = c->ny;
    size_t nc = (size_t)nx * ny;
    double dx = c->lx / nx, dy = c->ly / ny;
    double cD, ck, cS;
    if (c->ce_set == 1) { cD = 1.0; ck = 2.0; cS = 1.0; }
    else { cD = 2.0 / 3.0; ck = 5.0 / 2.0; cS = 2.0 / 3.0; }
    double twodx = 2.0 * dx, twody = 2.0 * dy;
    const double *ux = prim + nc, *uy = prim + 2 * nc, *T = prim + 3 * nc;
#define CI(ii, jj) ((size_t)orc_wrap(jj, ny) * nx + orc_wrap(ii, nx))
    for (int cell = 0; cell < nx * ny; ++cell) {
        int i = cell % nx, j = cell / nx;
        size_t ce = CI(i + 1, j), cw = CI(i - 1, j), cn = CI(i, j + 1), cs = CI(i, j - 1);
        double uxx = (ux[ce] - ux[cw]) / twodx;
        double uxy = (ux[cn] - ux[cs]) / twody;
        double uyx = (uy[ce] - uy[cw]) / twodx;
        double uyy = (uy[cn] - uy[cs]) / twody;
        double Tx = (T[ce] - T[cw]) / twodx;
        double Ty = (T[cn] - T[cs]) / twody;
        double div = uxx + uyy;
        double Dxx = (uxx + uxx) - cD * div;
        double Dxy = uxy + uyx;
        double Dyy = (uyy + uyy) - cD * div;
        double cv = eps[cell] / (c->tau * (1.0 - c->beta));
        double ke = ck * eps[cell];
        double kt2 = cS * ((ke * ke) / ((c->tau * c->tau) * T[cell]));
        double a11 = -(cv * Dxx) - kt2 * (Tx * Tx);
        double a12 = -(cv * Dxy) - kt2 * (Tx * Ty);
        double a22 = -(cv * Dyy) - kt2 * (Ty * Ty);
        double m = (a11 + a22) / 2.0;
        double h = (a11 - a22) / 2.0;
        double q = h * h + a12 * a12;
        if (lam_out) lam_out[cell] = fabs(m) + sqrt(q);
        /* |m| + sqrt(q) > eta  <=>  eta - |m| < 0  or  q > (eta - |m|)^2 */
        double dd = c->eta - fabs(m);
        int critS = (dd < 0.0) || (q > dd * dd);
        int critL = l1[cell] > c->delta;
        mask_new[cell] = (uint8_t)(critS || (mask_old[cell] && critL));
    }
#undef CI
}

/* --------------------------------------------------------------- driver */

/* Primitive variables (rho, ux, uy, T) from conserved U, both SoA [4][nc]. */
void orc_primitives(size_t nc, const double *U, double *prim)
{
    for (size_t q = 0; q < nc; ++q) {
        double rho = U[q], ux = U[nc + q] / rho, uy = U[2 * nc + q] / rho;
        double T = (U[3 * nc + q] - 0.5 * rho * (ux * ux + uy * uy)) / rho;
        prim[q] = rho; prim[nc + q] = ux; prim[2 * nc + q] = uy; prim[3 * nc + q] = T;
    }
}

/* Conserved U of one cell from its distribution (eq. Coupling_KinFlu). */
static void orc_conserved_of(const orc_cfg *c, const double *fc, size_t nc, size_t q, double *U)
{
    double mo[7];
    orc_moments(c, fc, mo);
    U[q] = mo[0];
    U[nc + q] = mo[0] * mo[1];
    U[2 * nc + q] = mo[0] * mo[2];
    U[3 * nc + q] = 0.5 * mo[0] * (mo[1] * mo[1] + mo[2] * mo[2]) + mo[0] * mo[3];
}

/* Fill f = Mhat(U) at one cell (eq. Coupling_FluKin). */
static int orc_fill_maxwellian(const orc_cfg *c, const double *U, size_t nc, size_t q, double *fc)
{
    double rho = U[q], ux = U[nc + q] / rho, uy = U[2 * nc + q] / rho;
    double T = (U[3 * nc + q] - 0.5 * rho * (ux * ux + uy * uy)) / rho;
    return orc_maxwellian_hat(c, rho, ux, uy, T, fc);
}

/* Stage coupling (Remark rem_coupling): every fluid cell carries the corrected
 * Maxwellian of its U as its distribution, every kinetic cell carries the
 * moments of its distribution as its U. */
static int orc_couple(const orc_cfg *c, const uint8_t *mask, double *f, double *U)
{
    size_t nc = (size_t)c->nx * c->ny, nv2 = (size_t)c->nv * c->nv;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long q = 0; q < (long)nc; ++q) {
        if (mask[q]) orc_conserved_of(c, f + q * nv2, nc, q, U);
        else bad |= orc_fill_maxwellian(c, U, nc, q, f + q * nv2) != 0;
    }
    return bad ? -1 : 0;
}

/* Regime update at the start of a step (Algorithm 1, first line of the loop):
 * indicator on the current moments, then the transitions of Sec. 3.3
 * (fluid -> kinetic: f = Mhat(U); kinetic -> fluid: U = moments(f), which the
 * coupling already holds).  l1 (size nc) receives the L1 distances used. */
int orc_regime_update(const orc_cfg *c, const double *f, const double *U, const double *eps,
                      uint8_t *mask, double *l1)
{
    size_t nc = (size_t)c->nx * c->ny, nv2 = (size_t)c->nv * c->nv;
    double *prim = (double *)malloc(4 * nc * sizeof(double));
    uint8_t *mnew = (uint8_t *)malloc(nc);
    orc_primitives(nc, U, prim);
#pragma omp parallel for schedule(static)
    for (long q = 0; q < (long)nc; ++q) l1[q] = mask[q] ? orc_l1_to_maxwellian(c, f + q * nv2) : 0.0;
    orc_indicator(c, prim, eps, l1, mask, mnew, NULL);
    memcpy(mask, mnew, nc);
    free(prim);
    free(mnew);
    return 0;
}

/* One time step of Algorithm 1 (high-order coupled domain decomposition) on
 * the current mask, with IMEX tableau (At, bt) explicit for transport and the
 * Euler flux (the Euler tableau equals the explicit one, Sec. 3.4.2) and
 * (A, b) implicit for the relaxation.  Both ARS tableaux have a zero first
 * implicit column and a zero first implicit weight, so the stage-1 source
 * never enters.
 *   Kinetic cells:  f^(i) = f^n - dt sum_j At_ij L(f^(j)) + dt sum_j A_ij S(f^(j)),
 *                   f^{n+1} = f^n - dt sum_i bt_i L(f^(i)) + dt sum_i b_i S(f^(i)),
 *                   S(f) = (tau/eps)(G[f] - f) (eqs. RKEI1, RKEI2);
 *   fluid cells:    U^(i) = U^n - dt sum_j At_ij Phi(U^(j)),
 *                   U^{n+1} = U^n - dt sum_i bt_i Phi(U^(i)) (eqs. RKEuler, RKEuler_2);
 *   coupling after every stage and after the final update (coupling = 0), or
 *   only after the final update (coupling = 1, the low-order-coupling variant).
 * f (nc*nv2) must already hold, at kinetic cells, the state at t^n; U (SoA)
 * holds U^n at every cell. */
int orc_step_once(const orc_cfg *c, double *f, double *U, const uint8_t *mask, const double *eps)
{
    size_t nc = (size_t)c->nx * c->ny, nv2 = (size_t)c->nv * c->nv, nf = nc * nv2;
    double At[9], bt[3], A[9], b[3];
    orc_tableau(c->scheme, At, bt, A, b);
    double dt = c->dt;
    double *fs[3], *Gs[3], *Ls[3], *Us[3], *Ps[3];
    for (int s = 0; s < 3; ++s) {
        fs[s] = (double *)calloc(nf, sizeof(double));
        Gs[s] = (double *)calloc(nf, sizeof(double));
        Ls[s] = (double *)calloc(nf, sizeof(double));
        Us[s] = (double *)calloc(4 * nc, sizeof(double));
        Ps[s] = (double *)calloc(4 * nc, sizeof(double));
    }
    double *fstar = (double *)malloc(nf * sizeof(double));
    int rc = 0;

    /* stage 1: f^(1) = f^n, U^(1) = U^n, with coupling */
    memcpy(fs[0], f, nf * sizeof(double));
    memcpy(Us[0], U, 4 * nc * sizeof(double));
    rc |= orc_couple(c, mask, fs[0], Us[0]);

    for (int i = 1; i < 3; ++i) {
        /* explicit operators of the previous stage */
        orc_transport(c, fs[i - 1], Ls[i - 1]);
        orc_euler_phi(c, Us[i - 1], Ps[i - 1]);
        /* fluid cells: Euler stage */
        for (size_t q = 0; q < nc; ++q) {
            if (mask[q]) continue;
            for (int m = 0; m < 4; ++m) {
                double s = U[m * nc + q];
                for (int j = 0; j < i; ++j) s -= dt * At[i * 3 + j] * Ps[j][m * nc + q];
                Us[i][m * nc + q] = s;
            }
        }
        /* kinetic cells: explicit part, then implicit relaxation */
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (long q = 0; q < (long)nc; ++q) {
            if (!mask[q]) continue;
            double tau_eps = c->tau / eps[q];
            for (size_t k = 0; k < nv2; ++k) {
                size_t idx = (size_t)q * nv2 + k;
                double s = f[idx];
                for (int j = 0; j < i; ++j) s -= dt * At[i * 3 + j] * Ls[j][idx];
                for (int j = 1; j < i; ++j)
                    s += dt * A[i * 3 + j] * tau_eps * (Gs[j][idx] - fs[j][idx]);
                fstar[idx] = s;
            }
            double lam = dt * A[i * 3 + i] * tau_eps;
            bad |= orc_relax_cell(c, fstar + (size_t)q * nv2, lam, fs[i] + (size_t)q * nv2,
                                  Gs[i] + (size_t)q * nv2, NULL) != 0;
        }
        rc |= bad ? -1 : 0;
        /* coupling of the stage */
        if (c->coupling == 0) {
            rc |= orc_couple(c, mask, fs[i], Us[i]);
        } else {
            /* low-order coupling: across the interface each solver keeps seeing
               the other one's values of t^n until the step ends */
            for (size_t q = 0; q < nc; ++q) {
                if (mask[q])
                    for (int m = 0; m < 4; ++m) Us[i][m * nc + q] = Us[0][m * nc + q];
                else
                    memcpy(fs[i] + q * nv2, fs[0] + q * nv2, nv2 * sizeof(double));
            }
        }
    }
    /* final update */
    orc_transport(c, fs[2], Ls[2]);
    orc_euler_phi(c, Us[2], Ps[2]);
    for (size_t q = 0; q < nc; ++q) {
        if (mask[q]) continue;
        for (int m = 0; m < 4; ++m) {
            double s = U[m * nc + q];
            for (int i = 0; i < 3; ++i) s -= dt * bt[i] * Ps[i][m * nc + q];
            U[m * nc + q] = s;
        }
    }
#pragma omp parallel for schedule(static)
    for (long q = 0; q < (long)nc; ++q) {
        if (!mask[q]) continue;
        double tau_eps = c->tau / eps[q];
        for (size_t k = 0; k < nv2; ++k) {
            size_t idx = (size_t)q * nv2 + k;
            double s = f[idx];
            for (int i = 0; i < 3; ++i) s -= dt * bt[i] * Ls[i][idx];
            for (int i = 1; i < 3; ++i) s += dt * b[i] * tau_eps * (Gs[i][idx] - fs[i][idx]);
            f[idx] = s;
        }
    }
    /* final coupling: kinetic U = moments(f^{n+1}) */
    for (size_t q = 0; q < nc; ++q)
        if (mask[q]) orc_conserved_of(c, f + q * nv2, nc, q, U);

    for (int s = 0; s < 3; ++s) {
        free(fs[s]); free(Gs[s]); free(Ls[s]); free(Us[s]); free(Ps[s]);
    }
    free(fstar);
    return rc;
}

/* nsteps of Algorithm 1.  update_regime = 1 runs the regime update at the
 * start of every step; 0 keeps the given mask (a fixed partition, as in the
 * order-of-accuracy test of Sec. 4.1.1).  l1 (nc) receives the last L1
 * distances.  Returns 0, or a negative value on a non-physical state. */
int orc_run(const orc_cfg *c, double *f, double *U, uint8_t *mask, const double *eps, double *l1,
            int nsteps, int update_regime)
{
    size_t nc = (size_t)c->nx * c->ny, nv2 = (size_t)c->nv * c->nv;
    uint8_t *old = (uint8_t *)malloc(nc);
    int rc = 0;
    for (int n = 0; n < nsteps && rc == 0; ++n) {
        if (update_regime) {
            memcpy(old, mask, nc);
            orc_regime_update(c, f, U, eps, mask, l1);
            for (size_t q = 0; q < nc; ++q)
                if (mask[q] && !old[q]) rc |= orc_fill_maxwellian(c, U, nc, q, f + q * nv2);
        }
        rc |= orc_step_once(c, f, U, mask, eps);
    }
    free(old);
    return rc;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
