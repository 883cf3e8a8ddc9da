"""Seeded synthetic initial data for the 2D2V ES-BGK workloads.

This module only draws and evaluates the initial macroscopic fields
(density, velocity, temperature, Knudsen number) on a cell-centred grid.  It
holds none of the method's arithmetic: the distribution functions are built
from these fields by the solver itself (and, independently, by the test
oracle), so both sides consume exactly the same arrays.

Every generator returns a dict of float64 arrays of length ``nx*ny`` in the
cell order ``i + nx*j`` (x fastest), evaluated at the cell centres
``x_i = (i + 1/2) lx/nx`` of the periodic box ``[0, lx] x [0, ly]``, plus the
grid / velocity-grid sizes the workload is defined with.

Workloads (shapes and value ranges follow the experiments of the ES-BGK
paper, arXiv 2512.03586, Sec. 4, and the synthetic configurations built on
them):

* ``smooth_density``  -- rho = 1 + A sin(2 pi x) sin(2 pi y), u = 0, T = 1,
  uniform eps (a smooth problem for the temporal-order study).
* ``riemann4``        -- four-quadrant Riemann problem, each quadrant a
  constant state with rho, T ~ U[0.5, 2] and |u| <= 1, drawn from a seed;
  log10 eps = -2 + 2 sin(2 pi x) sin(2 pi y)  (eps in [1e-4, 1]).
* ``shear_modes``     -- rho = 1 + 0.3 S1, T = 1 + 0.3 S2, S = sum of 8 seeded
  Fourier modes (|k|_inf <= 4) normalised to max |S| = 1;
  ux = 0.5 tanh((y - 1/2)/0.02), uy = 0; uniform eps.
* ``blast``           -- rho = 1, u = 0, T = 10 inside the disc of radius 0.1
  around the centre, T = 1 outside; log10 eps = -3 + 2 sin(2 pi x) sin(2 pi y).
* ``gaussian_bump``   -- the smooth bump of the paper's order test (Sec. 4.1.1):
  rho = 1 + 0.1 exp(-3 d^2), T = 0.3 (1 + 0.1 exp(-3 d^2)), u = 0.
"""
from __future__ import annotations

import numpy as np


def cell_centres(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0):
    x = (np.arange(nx) + 0.5) * (lx / nx)
    y = (np.arange(ny) + 0.5) * (ly / ny)
    X, Y = np.meshgrid(x, y, indexing="xy")     # [ny, nx] -> ravel gives i + nx*j
    return X.ravel(), Y.ravel()


def _pack(rho, ux, uy, T, eps, **meta):
    d = dict(rho=np.ascontiguousarray(rho, np.float64), ux=np.ascontiguousarray(ux, np.float64),
             uy=np.ascontiguousarray(uy, np.float64), T=np.ascontiguousarray(T, np.float64),
             eps=np.ascontiguousarray(eps, np.float64))
    d.update(meta)
    return d


def smooth_density(nx=32, ny=32, nv=16, vmax=8.0, amp=0.2, eps=1e-2):
    X, Y = cell_centres(nx, ny)
    rho = 1.0 + amp * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    z = np.zeros_like(X)
    return _pack(rho, z, z, np.ones_like(X), np.full_like(X, eps),
                 nx=nx, ny=ny, nv=nv, vmax=vmax, lx=1.0, ly=1.0)


def riemann4(nx=256, ny=256, nv=32, vmax=10.0, seed=0, log_eps_mean=-2.0, log_eps_amp=2.0):
    rng = np.random.default_rng(seed)
    rho_q = rng.uniform(0.5, 2.0, 4)
    T_q = rng.uniform(0.5, 2.0, 4)
    r_q = rng.uniform(0.0, 1.0, 4)
    phi_q = rng.uniform(0.0, 2 * np.pi, 4)
    X, Y = cell_centres(nx, ny)
    q = (X > 0.5).astype(int) + 2 * (Y > 0.5).astype(int)
    rho = rho_q[q]
    T = T_q[q]
    ux = (r_q * np.cos(phi_q))[q]
    uy = (r_q * np.sin(phi_q))[q]
    eps = 10.0 ** (log_eps_mean + log_eps_amp * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y))
    return _pack(rho, ux, uy, T, eps, nx=nx, ny=ny, nv=nv, vmax=vmax, lx=1.0, ly=1.0,
                 states=dict(rho=rho_q, T=T_q, ux=r_q * np.cos(phi_q), uy=r_q * np.sin(phi_q)))


def _fourier_field(rng, X, Y, nmodes=8, kmax=4):
    ks = []
    while len(ks) < nmodes:
        k = tuple(int(v) for v in rng.integers(-kmax, kmax + 1, 2))
        if k != (0, 0) and k not in ks and (-k[0], -k[1]) not in ks:
            ks.append(k)
    amps = rng.uniform(0.5, 1.0, nmodes)
    phases = rng.uniform(0.0, 2 * np.pi, nmodes)

    def ev(x, y):
        s = np.zeros_like(x)
        for (kx, ky), a, ph in zip(ks, amps, phases):
            s += a * np.cos(2 * np.pi * (kx * x + ky * y) + ph)
        return s

    # normalisation on a fixed fine grid, so that every resolution samples the same field
    xf, yf = cell_centres(512, 512)
    norm = np.max(np.abs(ev(xf, yf)))
    return ev(X, Y) / norm


def shear_modes(nx=512, ny=512, nv=48, vmax=8.0, seed=0, amp=0.3, eps=1e-3, width=0.02):
    rng = np.random.default_rng(seed)
    X, Y = cell_centres(nx, ny)
    S1 = _fourier_field(rng, X, Y)
    S2 = _fourier_field(rng, X, Y)
    rho = 1.0 + amp * S1
    T = 1.0 + amp * S2
    ux = 0.5 * np.tanh((Y - 0.5) / width)
    return _pack(rho, ux, np.zeros_like(X), T, np.full_like(X, eps),
                 nx=nx, ny=ny, nv=nv, vmax=vmax, lx=1.0, ly=1.0)


def blast(nx=1024, ny=1024, nv=64, vmax=20.0, radius=0.1, T_in=10.0,
          log_eps_mean=-3.0, log_eps_amp=2.0):
    X, Y = cell_centres(nx, ny)
    inside = (X - 0.5) ** 2 + (Y - 0.5) ** 2 < radius ** 2
    T = np.where(inside, T_in, 1.0)
    eps = 10.0 ** (log_eps_mean + log_eps_amp * np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y))
    z = np.zeros_like(X)
    return _pack(np.ones_like(X), z, z, T, eps, nx=nx, ny=ny, nv=nv, vmax=vmax, lx=1.0, ly=1.0)


def gaussian_bump(nx=90, ny=90, nv=32, vmax=5.0, L=6.0, eps=1e-2, lam=3.0):
    X, Y = cell_centres(nx, ny, L, L)
    d2 = (X - L / 2) ** 2 + (Y - L / 2) ** 2
    g = np.exp(-lam * d2)
    z = np.zeros_like(X)
    return _pack(1.0 + 0.1 * g, z, z, 0.3 * (1.0 + 0.1 * g), np.full_like(X, eps),
                 nx=nx, ny=ny, nv=nv, vmax=vmax, lx=L, ly=L)


def random_partition(nc: int, frac: float = 0.5, seed: int = 0) -> np.ndarray:
    """Fixed random kinetic/fluid partition (1 = kinetic), as in the paper's
    order-of-accuracy test where each cell's regime is drawn once at t = 0."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(size=nc) < frac).astype(np.uint8)


def random_distribution(nc: int, nv2: int, seed: int = 0, lo: float = 0.05, hi: float = 1.0):
    """Strictly positive random phase-space values (for operator-level tests that
    need a distribution far from equilibrium)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (nc, nv2))
