"""Independent NumPy brute force of the coupled IMEX ES-BGK step, for tiny grids.

Used only to pin the oracle.  It shares nothing with ``oracle/``: velocity
nodes come from ``np.linspace``, the anisotropic Gaussian from
``scipy.stats.multivariate_normal``, stencils from ``np.roll``, and every
implicit stage is solved by Newton's method on the full nonlinear system
``f = f* + lam (G[f] - f)`` (finite-difference Jacobian) instead of the closed
form the oracle uses.  Arrays: f[ny, nx, nv2], U[4, ny, nx].
"""
from __future__ import annotations

import numpy as np
from scipy.stats import multivariate_normal


class BF:
    def __init__(self, nx, ny, nv, vmax, lx=1.0, ly=1.0, beta=-0.5, tau=1.0, dt=None,
                 scheme=1, recon=1, correction=True, cfl=0.5):
        self.nx, self.ny, self.nv, self.V = nx, ny, nv, vmax
        self.dx, self.dy = lx / nx, ly / ny
        self.beta, self.tau = beta, tau
        self.dt = dt if dt else cfl * min(self.dx, self.dy) / vmax
        self.recon, self.correction = recon, correction
        self.dv = 2 * vmax / nv
        self.w = self.dv ** 2
        v = np.linspace(-vmax + self.dv / 2, vmax - self.dv / 2, nv)
        VX, VY = np.meshgrid(v, v, indexing="xy")
        self.vx, self.vy = VX.ravel(), VY.ravel()
        self.pts = np.stack([self.vx, self.vy], axis=1)
        if scheme == 1:
            a = (3 + np.sqrt(3)) / 6
            self.At = np.array([[0, 0, 0], [a, 0, 0], [a - 1, 2 - 2 * a, 0]])
            self.bt = np.array([0, .5, .5])
            self.A = np.array([[0, 0, 0], [0, a, 0], [0, 1 - 2 * a, a]])
            self.b = np.array([0, .5, .5])
        else:
            g = 1 - 1 / np.sqrt(2); d = 1 - 1 / (2 * g)
            self.At = np.array([[0, 0, 0], [g, 0, 0], [d, 1 - d, 0]])
            self.bt = np.array([d, 1 - d, 0])
            self.A = np.array([[0, 0, 0], [0, g, 0], [0, 1 - g, g]])
            self.b = np.array([0, 1 - g, g])

    # ---- velocity space
    def moments(self, fc):
        rho = self.w * fc.sum()
        u = self.w * (self.pts * fc[:, None]).sum(0) / rho
        xi = self.pts - u
        Th = self.w * np.einsum("k,ki,kj->ij", fc, xi, xi) / rho
        return rho, u, np.trace(Th) / 2, Th

    def gauss(self, rho, u, T, Tt):
        g = rho * multivariate_normal(mean=u, cov=Tt).pdf(self.pts)
        if self.correction:
            xi = (self.pts - u) / np.sqrt(T)
            psi = np.stack([np.ones(len(g)), xi[:, 0], xi[:, 1], xi[:, 0] ** 2,
                            xi[:, 0] * xi[:, 1], xi[:, 1] ** 2], axis=1)
            Gram = self.w * np.einsum("k,km,kn->mn", g, psi, psi)
            t = rho * np.array([1, 0, 0, Tt[0, 0] / T, Tt[0, 1] / T, Tt[1, 1] / T])
            g = g * (psi @ np.linalg.solve(Gram, t))
        return g

    def G_of(self, fc):
        rho, u, T, Th = self.moments(fc)
        Tt = (1 - self.beta) * T * np.eye(2) + self.beta * Th
        return self.gauss(rho, u, T, Tt)

    def maxwell(self, rho, u, T):
        return self.gauss(rho, np.asarray(u, float), T, T * np.eye(2))

    def solve_implicit(self, fstar, lam, iters=30):
        """Newton on R(f) = f - fstar - lam (G[f] - f) = 0."""
        f = fstar.copy()
        n = len(f)
        for _ in range(iters):
            R = f - fstar - lam * (self.G_of(f) - f)
            if np.max(np.abs(R)) < 1e-15 * np.max(np.abs(fstar)):
                break
            J = np.empty((n, n))
            for m in range(n):
                h = 1e-7 * max(abs(f[m]), 1e-3)
                e = np.zeros(n); e[m] = h
                Rp = (f + e) - fstar - lam * (self.G_of(f + e) - (f + e))
                Rm = (f - e) - fstar - lam * (self.G_of(f - e) - (f - e))
                J[:, m] = (Rp - Rm) / (2 * h)
            f = f - np.linalg.solve(J, R)
        return f

    # ---- space
    @staticmethod
    def _mm(a, b):
        return np.where(a * b <= 0, 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)))

    def _faces(self, q, axis):
        """Left / right states at faces (i+1/2) along axis (periodic)."""
        if self.recon == 1:
            s = self._mm(q - np.roll(q, 1, axis), np.roll(q, -1, axis) - q)
        else:
            s = np.zeros_like(q)
        qL = q + 0.5 * s
        qR = np.roll(q - 0.5 * s, -1, axis)
        return qL, qR

    def transport(self, f):
        out = np.zeros_like(f)
        for axis, v, h in ((1, self.vx, self.dx), (0, self.vy, self.dy)):
            fL, fR = self._faces(f, axis)
            F = np.maximum(v, 0) * fL + np.minimum(v, 0) * fR
            out += (F - np.roll(F, 1, axis)) / h
        return out

    @staticmethod
    def flux(U, d):
        rho, mx, my, E = U
        ux, uy = mx / rho, my / rho
        P = E - 0.5 * rho * (ux ** 2 + uy ** 2)
        un = ux if d == 0 else uy
        return np.stack([rho * un, mx * un + (P if d == 0 else 0), my * un + (P if d == 1 else 0),
                         un * (E + P)])

    @staticmethod
    def speed(U, d):
        rho, mx, my, E = U
        ux, uy = mx / rho, my / rho
        P = E - 0.5 * rho * (ux ** 2 + uy ** 2)
        return np.abs(ux if d == 0 else uy) + np.sqrt(2 * P / rho)

    def phi(self, U):
        out = np.zeros_like(U)
        for d, axis, h in ((0, 2, self.dx), (1, 1, self.dy)):
            UL, UR = self._faces(U, axis)
            a = np.maximum(self.speed(UL, d), self.speed(UR, d))
            F = 0.5 * (self.flux(UL, d) + self.flux(UR, d)) - 0.5 * a * (UR - UL)
            out += (F - np.roll(F, 1, axis)) / h
        return out

    # ---- coupled step (Algorithm 1 with coupling at every stage)
    def conserved_of(self, fc):
        rho, u, T, _ = self.moments(fc)
        return np.array([rho, rho * u[0], rho * u[1], 0.5 * rho * (u @ u) + rho * T])

    def prim(self, Uc):
        rho = Uc[0]; u = Uc[1:3] / rho
        return rho, u, (Uc[3] - 0.5 * rho * (u @ u)) / rho

    def couple(self, mask, f, U):
        f = f.copy(); U = U.copy()
        for j in range(self.ny):
            for i in range(self.nx):
                if mask[j, i]:
                    U[:, j, i] = self.conserved_of(f[j, i])
                else:
                    f[j, i] = self.maxwell(*self.prim(U[:, j, i]))
        return f, U

    def step(self, f, U, mask, eps):
        """One step; f[ny,nx,nv2], U[4,ny,nx], mask/eps [ny,nx]. Returns (f, U)."""
        dt = self.dt
        te = self.tau / eps
        fs, Us, Gs = [None] * 3, [None] * 3, [None] * 3
        fs[0], Us[0] = self.couple(mask, f, U)
        for i in (1, 2):
            Ls = [self.transport(fs[j]) for j in range(i)]
            Ph = [self.phi(Us[j]) for j in range(i)]
            Un = U - dt * sum(self.At[i, j] * Ph[j] for j in range(i))
            fi = np.zeros_like(f); Gi = np.zeros_like(f)
            for jj in range(self.ny):
                for ii in range(self.nx):
                    if not mask[jj, ii]:
                        continue
                    fst = f[jj, ii] - dt * sum(self.At[i, j] * Ls[j][jj, ii] for j in range(i))
                    for j in range(1, i):
                        fst = fst + dt * self.A[i, j] * te[jj, ii] * (Gs[j][jj, ii] - fs[j][jj, ii])
                    lam = dt * self.A[i, i] * te[jj, ii]
                    fi[jj, ii] = self.solve_implicit(fst, lam)
                    Gi[jj, ii] = self.G_of(fi[jj, ii])
            Un = np.where(mask[None], U, Un)
            fs[i], Us[i] = self.couple(mask, fi, Un)
            Gs[i] = Gi
        Ls = [self.transport(fs[i]) for i in range(3)]
        Ph = [self.phi(Us[i]) for i in range(3)]
        Unew = U - dt * sum(self.bt[i] * Ph[i] for i in range(3))
        fnew = f - dt * sum(self.bt[i] * Ls[i] for i in range(3))
        for i in (1, 2):
            fnew = fnew + dt * self.b[i] * te[..., None] * (Gs[i] - fs[i])
        fnew = np.where(mask[..., None], fnew, f)
        Unew = np.where(mask[None], U, Unew)
        for jj in range(self.ny):
            for ii in range(self.nx):
                if mask[jj, ii]:
                    Unew[:, jj, ii] = self.conserved_of(fnew[jj, ii])
        return fnew, Unew
