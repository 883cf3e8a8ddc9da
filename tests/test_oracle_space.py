"""Pins of the oracle's spatial operators: kinetic transport L(f) and the Euler
divergence Phi(U), plus the regime indicator.

Checked against telescoping sums, exact shifts, linear reproduction, the
kinetic moments of a Maxwellian flux, the spectral radius of the Euler flux
Jacobian, numpy eigenvalues and an independent np.roll implementation.
"""
import numpy as np
import pytest

from bruteforce import BF


def prob(orc, nx=6, ny=5, nv=4, vmax=2.0, **kw):
    return orc.Problem(nx=nx, ny=ny, nv=nv, vmax=vmax, **kw)


# ------------------------------------------------------------------ transport

@pytest.mark.parametrize("recon", [0, 1])
def test_transport_of_constant_is_zero(orc, recon):
    p = prob(orc, recon=recon)
    f = np.tile(np.random.default_rng(0).uniform(0.1, 1, p.nv2), (p.nc, 1))
    assert np.max(np.abs(orc.transport(p, f))) < 1e-12


@pytest.mark.parametrize("recon", [0, 1])
def test_transport_telescopes_on_periodic_grid(orc, recon):
    p = prob(orc, recon=recon)
    f = np.random.default_rng(1).uniform(0.1, 1, (p.nc, p.nv2))
    L = orc.transport(p, f)
    assert np.max(np.abs(L.sum(0))) < 1e-11 * np.abs(L).sum(0).max()


def test_upwind_at_courant_one_is_exact_shift(orc):
    """First-order upwind, forward Euler with |v| dt = dx: f moves one cell downwind."""
    p = prob(orc, nx=7, ny=3, nv=4, vmax=2.0, recon=0)
    rng = np.random.default_rng(2)
    prof = rng.uniform(0.1, 1.0, p.nx)
    f = np.repeat(np.tile(prof, p.ny)[:, None], p.nv2, axis=1)   # varies in x only
    L = orc.transport(p, f)
    vx, _ = orc.velocity_nodes(p)
    dx = p.lx / p.nx
    for k in range(p.nv2):
        new = (f[:, k] - dx / abs(vx[k]) * L[:, k]).reshape(p.ny, p.nx)
        shift = 1 if vx[k] > 0 else -1
        np.testing.assert_allclose(new, np.roll(prof, shift)[None].repeat(p.ny, 0), atol=1e-14)


def test_minmod_reproduces_linear_data_in_interior(orc):
    p = prob(orc, nx=12, ny=2, nv=4, vmax=2.0, recon=1)
    X = (np.arange(p.nx) + 0.5) / p.nx
    slope = 0.8
    f = np.repeat(np.tile(1.0 + slope * X, p.ny)[:, None], p.nv2, axis=1)
    L = orc.transport(p, f).reshape(p.ny, p.nx, p.nv2)
    vx, _ = orc.velocity_nodes(p)
    # interior cells (two away from the periodic seam)
    np.testing.assert_allclose(L[:, 2:-2, :], np.broadcast_to(vx * slope, L[:, 2:-2, :].shape),
                               rtol=1e-12, atol=1e-12)


def test_minmod_flattens_at_extremum(orc):
    """A local maximum gets zero slope: both face values equal the cell value (TVD)."""
    p = prob(orc, nx=7, ny=1, nv=2, vmax=1.0, recon=1)   # vx = +-0.5
    prof = np.array([0, 0, 1.0, 3.0, 1.0, 0, 0])
    f = np.repeat(prof[:, None], p.nv2, axis=1)
    L = orc.transport(p, f)
    vx, _ = orc.velocity_nodes(p)
    k = int(np.argmax(vx))                 # vx > 0 (the y part vanishes: ny = 1)
    dx = p.lx / p.nx
    # cell 3 (maximum): F_{3+1/2} = v * 3 (flat), F_{3-1/2} = v * (1 + minmod(1, 2)/2) = 1.5 v
    assert L[3, k] == pytest.approx(vx[k] * (3.0 - 1.5) / dx, rel=1e-13)


@pytest.mark.parametrize("recon", [0, 1])
def test_transport_matches_numpy_roll_bruteforce(orc, recon):
    p = prob(orc, nx=4, ny=4, nv=4, vmax=2.0, recon=recon)
    bf = BF(4, 4, 4, 2.0, recon=recon)
    f = np.random.default_rng(3).uniform(0.1, 1, (p.nc, p.nv2))
    ref = bf.transport(f.reshape(p.ny, p.nx, p.nv2)).reshape(p.nc, p.nv2)
    np.testing.assert_allclose(orc.transport(p, f), ref, rtol=1e-13, atol=1e-12)


# ---------------------------------------------------------------------- Euler

def test_euler_flux_is_kinetic_flux_of_maxwellian(orc):
    """F(U) equals the velocity moments (1, v, |v|^2/2) of v_n * M on a fine grid
    (compressible Euler limit of Sec. 2 with gamma = 2, P = rho T)."""
    p = orc.Problem(nx=1, ny=1, nv=96, vmax=14.0)
    vx, vy = orc.velocity_nodes(p)
    w = (2 * p.vmax / p.nv) ** 2
    rho, ux, uy, T = 1.3, 0.6, -0.4, 1.2
    m = orc.maxwellian(p, rho, ux, uy, T)
    U = orc.conserved(rho, ux, uy, T)
    for d, vn in ((0, vx), (1, vy)):
        kin = w * np.array([(vn * m).sum(), (vn * vx * m).sum(), (vn * vy * m).sum(),
                            (vn * 0.5 * (vx ** 2 + vy ** 2) * m).sum()])
        np.testing.assert_allclose(orc.euler_flux(U, d), kin, rtol=1e-10)


def test_rusanov_consistency_and_speed_is_spectral_radius(orc):
    rng = np.random.default_rng(4)
    for _ in range(5):
        rho, ux, uy, T = rng.uniform(0.5, 2), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.5, 2)
        U = orc.conserved(rho, ux, uy, T)
        for d in (0, 1):
            np.testing.assert_allclose(orc.rusanov(U, U, d), orc.euler_flux(U, d), rtol=1e-14)
            # dissipation coefficient = spectral radius of dF/dU (finite differences)
            J = np.empty((4, 4))
            for m in range(4):
                e = np.zeros(4); e[m] = 1e-6 * max(1.0, abs(U[m]))
                J[:, m] = (orc.euler_flux(U + e, d) - orc.euler_flux(U - e, d)) / (2 * e[m])
            srad = np.max(np.abs(np.linalg.eigvals(J)))
            dU = np.array([1e-3, -2e-3, 1.5e-3, 1e-3])
            Fh = orc.rusanov(U, U + dU, d)
            avg = 0.5 * (orc.euler_flux(U, d) + orc.euler_flux(U + dU, d))
            a = -np.dot(Fh - avg, dU) / (0.5 * np.dot(dU, dU))
            assert a == pytest.approx(srad, rel=2e-3)


@pytest.mark.parametrize("recon", [0, 1])
def test_euler_phi_conserves_and_matches_bruteforce(orc, recon):
    p = prob(orc, nx=5, ny=4, recon=recon)
    rng = np.random.default_rng(5)
    U = orc.conserved(rng.uniform(0.5, 2, p.nc), rng.uniform(-1, 1, p.nc),
                      rng.uniform(-1, 1, p.nc), rng.uniform(0.5, 2, p.nc))
    Phi = orc.euler_phi(p, U)
    assert np.max(np.abs(Phi.sum(1))) < 1e-11 * np.abs(Phi).sum()
    bf = BF(5, 4, 4, 2.0, recon=recon)
    ref = bf.phi(U.reshape(4, p.ny, p.nx)).reshape(4, p.nc)
    np.testing.assert_allclose(Phi, ref, rtol=1e-12, atol=1e-11)
    Uc = np.tile(U[:, :1], (1, p.nc))
    assert np.max(np.abs(orc.euler_phi(p, Uc))) < 1e-12


# ------------------------------------------------------------------ indicator

def _np_lambda(p, prim, eps, cD, ck, cS):
    """Largest |eigenvalue| of S1 - I via numpy eigvalsh (independent)."""
    rho, ux, uy, T = (prim[q].reshape(p.ny, p.nx) for q in range(4))
    dx, dy = p.lx / p.nx, p.ly / p.ny
    gx = lambda q: (np.roll(q, -1, 1) - np.roll(q, 1, 1)) / (2 * dx)
    gy = lambda q: (np.roll(q, -1, 0) - np.roll(q, 1, 0)) / (2 * dy)
    out = np.empty(p.nc)
    e = eps.reshape(p.ny, p.nx)
    G = np.stack([[gx(ux), gy(ux)], [gx(uy), gy(uy)]])       # G[a,b] = d u_a / d x_b
    gT = np.stack([gx(T), gy(T)])
    for j in range(p.ny):
        for i in range(p.nx):
            g = G[:, :, j, i]
            D = g + g.T - cD * np.trace(g) * np.eye(2)
            mu = 1 / (p.tau * (1 - p.beta))
            kap = ck / (p.tau * np.sqrt(T[j, i]))
            A = -e[j, i] * mu * D - cS * (e[j, i] * kap) ** 2 * np.outer(gT[:, j, i], gT[:, j, i])
            out[i + p.nx * j] = np.max(np.abs(np.linalg.eigvalsh(A)))
    return out


@pytest.mark.parametrize("ce_set,consts", [(0, (2 / 3, 5 / 2, 2 / 3)), (1, (1.0, 2.0, 1.0))])
def test_indicator_eigenvalue_matches_numpy(orc, ce_set, consts):
    p = prob(orc, nx=7, ny=6, ce_set=ce_set)
    rng = np.random.default_rng(6)
    prim = np.stack([rng.uniform(0.5, 2, p.nc), rng.uniform(-1, 1, p.nc),
                     rng.uniform(-1, 1, p.nc), rng.uniform(0.5, 2, p.nc)])
    eps = 10 ** rng.uniform(-4, 0, p.nc)
    _, lam = orc.indicator(p, prim, eps, np.zeros(p.nc), np.zeros(p.nc, np.uint8), return_lambda=True)
    np.testing.assert_allclose(lam, _np_lambda(p, prim, eps, *consts), rtol=1e-12)


def test_indicator_eps_zero_gives_all_fluid(orc):
    """eps = 0 => S1 = S0 = I => the whole domain is hydrodynamic (Sec. 3.6)."""
    p = prob(orc, nx=6, ny=6)
    rng = np.random.default_rng(7)
    prim = np.stack([rng.uniform(0.5, 2, p.nc), rng.uniform(-3, 3, p.nc),
                     rng.uniform(-3, 3, p.nc), rng.uniform(0.2, 5, p.nc)])
    m = orc.indicator(p, prim, np.zeros(p.nc), np.zeros(p.nc), np.zeros(p.nc, np.uint8))
    assert m.sum() == 0


def test_indicator_uniform_state_is_fluid(orc):
    p = prob(orc, nx=5, ny=5)
    prim = np.tile(np.array([[1.2], [0.3], [-0.1], [0.9]]), (1, p.nc))
    _, lam = orc.indicator(p, prim, np.ones(p.nc), np.zeros(p.nc), np.zeros(p.nc, np.uint8),
                           return_lambda=True)
    assert np.all(lam == 0.0)


def test_indicator_hysteresis_truth_table(orc):
    """fluid->kinetic iff crit_S; kinetic->fluid iff not crit_S and L1 <= delta."""
    p = prob(orc, nx=8, ny=1, eta=1e-2, delta=1e-3)
    # gradients only in T along x: lam_i grows with |dT/dx|
    T = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    prim = np.stack([np.ones(8), np.zeros(8), np.zeros(8), T])
    eps = np.full(8, 1e-2)
    _, lam0 = orc.indicator(p, prim, eps, np.zeros(8), np.zeros(8, np.uint8), return_lambda=True)
    assert np.all(lam0 == 0)
    eps_hi = np.full(8, 1e6)       # no gradient: never crit_S, whatever eps
    for old in (0, 1):
        for l1 in (0.0, 5e-4, 2e-3):
            m = orc.indicator(p, prim, eps_hi, np.full(8, l1), np.full(8, old, np.uint8))
            assert np.all(m == (1 if (old and l1 > 1e-3) else 0))
    # a temperature jump makes crit_S true regardless of the history
    T2 = T.copy(); T2[4] = 3.0
    prim2 = np.stack([np.ones(8), np.zeros(8), np.zeros(8), T2])
    for old in (0, 1):
        m = orc.indicator(p, prim2, np.full(8, 1.0), np.zeros(8), np.full(8, old, np.uint8))
        assert m[3] == 1 and m[5] == 1 and m[0] == old * 0


def test_indicator_temperature_term_constants(orc):
    """u = 0, T gradient only: lam = cS (ck eps |dT|/(tau sqrt T))^2 (paper constants 2/3, 5/2)."""
    p = prob(orc, nx=6, ny=1, ce_set=0)
    T = np.array([1.0, 1.0, 1.2, 1.0, 1.0, 1.0])
    prim = np.stack([np.ones(6), np.zeros(6), np.zeros(6), T])
    eps = np.full(6, 0.1)
    _, lam = orc.indicator(p, prim, eps, np.zeros(6), np.zeros(6, np.uint8), return_lambda=True)
    dTdx = (1.2 - 1.0) / (2 * p.lx / p.nx)          # at cell 1 (neighbours 0 and 2)
    expect = (2 / 3) * (2.5 * 0.1 * dTdx / 1.0) ** 2
    assert lam[1] == pytest.approx(expect, rel=1e-13)
