"""Pins of the oracle's velocity-space pieces: moments, Maxwellian, the ES-BGK
Gaussian, its discrete-conservation correction and the implicit relaxation.

Each test checks the oracle against something it does not contain: a closed
form, a library routine (scipy's multivariate normal), an invariant of the
paper, or an independent brute force (Newton on the nonlinear implicit
equation).
"""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

from bruteforce import BF


def grid(orc, nv=48, vmax=10.0, **kw):
    return orc.Problem(nx=1, ny=1, nv=nv, vmax=vmax, **kw)


def np_moments(p, f):
    """Moments by direct numpy quadrature on linspace nodes (independent nodes)."""
    dv = 2 * p.vmax / p.nv
    v = np.linspace(-p.vmax + dv / 2, p.vmax - dv / 2, p.nv)
    VX, VY = np.meshgrid(v, v, indexing="xy")
    vx, vy = VX.ravel(), VY.ravel()
    w = dv * dv
    rho = w * f.sum()
    ux, uy = w * (vx * f).sum() / rho, w * (vy * f).sum() / rho
    th = np.array([[(w * (vx - ux) ** 2 * f).sum(), (w * (vx - ux) * (vy - uy) * f).sum()],
                   [(w * (vx - ux) * (vy - uy) * f).sum(), (w * (vy - uy) ** 2 * f).sum()]]) / rho
    return rho, ux, uy, np.trace(th) / 2, th


# Sec. 3.2: node placement and quadrature weight -------------------------------------------

def test_velocity_nodes_are_midpoints(orc):
    p = grid(orc, nv=8, vmax=4.0)
    vx, vy = orc.velocity_nodes(p)
    v = np.linspace(-3.5, 3.5, 8)
    np.testing.assert_array_equal(vx.reshape(8, 8)[0], v)     # x fastest
    np.testing.assert_array_equal(vy.reshape(8, 8)[:, 0], v)


def test_moments_match_numpy_quadrature(orc):
    rng = np.random.default_rng(1)
    for nv in (4, 12, 32):
        p = grid(orc, nv=nv, vmax=5.0)
        f = rng.uniform(0.1, 1.0, p.nv2)
        mo = orc.moments(p, f)
        rho, ux, uy, T, th = np_moments(p, f)
        np.testing.assert_allclose(mo[:4], [rho, ux, uy, T], rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(mo[4:], [th[0, 0], th[0, 1], th[1, 1]], rtol=1e-12, atol=1e-14)


# H3: the sampled Maxwellian carries (rho, u, T) up to the quadrature error ----------------

@pytest.mark.parametrize("T", [0.5, 1.5])
def test_maxwellian_moments_within_quadrature_bound(orc, T):
    p = grid(orc, nv=48, vmax=10.0)
    rho, ux, uy = 1.3, 0.4, -0.7
    m = orc.maxwellian(p, rho, ux, uy, T)
    mo = orc.moments(p, m)
    dv = 2 * p.vmax / p.nv
    alias = 2 * np.exp(-2 * np.pi ** 2 * T / dv ** 2)            # Poisson summation
    trunc = np.exp(-(p.vmax - 1.0) ** 2 / (2 * T)) * 10           # tail beyond the box
    tol = max(alias, trunc) + 1e-13
    np.testing.assert_allclose(mo[:4], [rho, ux, uy, T], rtol=tol, atol=tol)
    np.testing.assert_allclose(mo[4:], [T, 0.0, T], rtol=tol, atol=tol)


def test_maxwellian_matches_scipy(orc):
    p = grid(orc, nv=16, vmax=6.0)
    vx, vy = orc.velocity_nodes(p)
    m = orc.maxwellian(p, 0.8, 0.3, 0.2, 1.1)
    ref = 0.8 * multivariate_normal(mean=[0.3, 0.2], cov=1.1 * np.eye(2)).pdf(np.c_[vx, vy])
    np.testing.assert_allclose(m, ref, rtol=1e-13)


# Sec. 2: anisotropic Gaussian G ---------------------------------------------------------

def test_gaussian_tilde_matches_scipy_anisotropic(orc):
    p = grid(orc, nv=20, vmax=6.0)
    vx, vy = orc.velocity_nodes(p)
    cov = np.array([[1.4, 0.35], [0.35, 0.6]])
    g = orc.gaussian_tilde(p, 1.7, -0.4, 0.25, cov[0, 0], cov[0, 1], cov[1, 1])
    ref = 1.7 * multivariate_normal(mean=[-0.4, 0.25], cov=cov).pdf(np.c_[vx, vy])
    np.testing.assert_allclose(g, ref, rtol=1e-12)


def test_gaussian_moments_are_es_tensor_fine_grid(orc):
    """On a resolved grid the sampled Gaussian's Theta is the tensor it was built from."""
    p = grid(orc, nv=64, vmax=10.0, correction=0)
    g = orc.gaussian_tilde(p, 1.1, 0.3, -0.2, 1.3, -0.4, 0.7)
    mo = orc.moments(p, g)
    np.testing.assert_allclose(mo[[0, 1, 2]], [1.1, 0.3, -0.2], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(mo[4:], [1.3, -0.4, 0.7], rtol=1e-10, atol=1e-11)


def test_corrected_gaussian_has_exact_discrete_moments(orc):
    """Under-resolved grid (dv = 1, T = 0.6): the sampled Gaussian misses its moments
    by ~1e-5, the corrected one hits (rho, u, Tt) to roundoff."""
    p = grid(orc, nv=8, vmax=4.0)
    rho, ux, uy, T = 0.9, 0.2, -0.3, 0.6
    th = np.array([[0.8, 0.15], [0.15, 0.4]])
    tt = (1 - p.beta) * T * np.eye(2) + p.beta * th
    g0 = orc.gaussian_tilde(p, rho, ux, uy, tt[0, 0], tt[0, 1], tt[1, 1])
    g = orc.gaussian_hat(p, rho, ux, uy, T, tt[0, 0], tt[0, 1], tt[1, 1])
    r0, ux0, uy0, _, th0 = np_moments(p, g0)
    assert abs(r0 - rho) > 1e-7              # the correction has work to do
    r1, ux1, uy1, T1, th1 = np_moments(p, g)
    np.testing.assert_allclose([r1, ux1, uy1], [rho, ux, uy], rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(th1, tt, rtol=1e-12, atol=1e-13)


def test_correction_off_returns_sampled_gaussian(orc):
    p = grid(orc, nv=8, vmax=4.0, correction=0)
    g0 = orc.gaussian_tilde(p, 1.0, 0.1, 0.0, 0.9, 0.1, 1.1)
    g, c = orc.gaussian_hat(p, 1.0, 0.1, 0.0, 1.0, 0.9, 0.1, 1.1, return_coef=True)
    np.testing.assert_array_equal(g, g0)
    np.testing.assert_array_equal(c, [1, 0, 0, 0, 0, 0])


def test_G_of_maxwellian_is_maxwellian(orc):
    """Theta = T I  =>  Tt = T I  =>  G[M] = M (Sec. 2)."""
    p = grid(orc, nv=12, vmax=6.0)
    m = orc.maxwellian_hat(p, 1.2, -0.5, 0.3, 0.8)
    np.testing.assert_allclose(orc.gaussian_of(p, m), m, rtol=1e-12, atol=1e-15)


def test_beta_zero_gives_bgk_maxwellian(orc):
    """beta = 0 reduces the ES-BGK Gaussian to the BGK Maxwellian of f's moments."""
    p = grid(orc, nv=16, vmax=6.0, beta=0.0)
    f = np.random.default_rng(3).uniform(0.05, 1.0, p.nv2)
    mo = orc.moments(p, f)
    np.testing.assert_allclose(orc.gaussian_of(p, f), orc.maxwellian_hat(p, *mo[:4]),
                               rtol=1e-12, atol=1e-15)


def test_es_tensor_uses_beta(orc):
    """Tt = (1-beta) T I + beta Theta: the Gaussian's Theta must follow beta."""
    p = grid(orc, nv=48, vmax=10.0)
    vx, vy = orc.velocity_nodes(p)
    th = np.array([[1.6, 0.3], [0.3, 0.4]])
    f = multivariate_normal(mean=[0.1, 0.2], cov=th).pdf(np.c_[vx, vy])
    mo = orc.moments(p, f)
    T = mo[3]
    th_f = np.array([[mo[4], mo[5]], [mo[5], mo[6]]])
    for beta in (-0.5, 0.0, 0.5):
        p.beta = beta
        g = orc.gaussian_of(p, f)
        _, _, _, _, thg = np_moments(p, g)
        np.testing.assert_allclose(thg, (1 - beta) * T * np.eye(2) + beta * th_f, rtol=1e-11, atol=1e-12)


# Relaxation (implicit stage) ------------------------------------------------------------

def test_relaxation_conserves_mass_momentum_energy(orc):
    """H1: the implicit stage changes no conserved moment."""
    p = grid(orc, nv=10, vmax=5.0)
    rng = np.random.default_rng(5)
    vx, vy = orc.velocity_nodes(p)
    for lam in (1e-3, 0.7, 50.0):
        fs = rng.uniform(0.02, 1.0, p.nv2)
        f, _, _ = orc.relax_cell(p, fs, lam)
        w = (2 * p.vmax / p.nv) ** 2
        for phi in (np.ones_like(vx), vx, vy, 0.5 * (vx ** 2 + vy ** 2)):
            a, b = w * (phi * fs).sum(), w * (phi * f).sum()
            assert abs(a - b) <= 1e-13 * (abs(a) + w * (np.abs(phi) * fs).sum())


def test_relaxation_closed_form_equals_newton_bruteforce(orc):
    """The closed form solves f = f* + lam (G[f] - f): compare with Newton on the
    full nonlinear system (4x4 velocities, scipy Gaussian)."""
    p = grid(orc, nv=4, vmax=2.0)
    bf = BF(1, 1, 4, 2.0)
    rng = np.random.default_rng(11)
    for lam in (0.05, 1.0, 20.0):
        fs = rng.uniform(0.05, 0.3, 16)
        f_closed, _, _ = orc.relax_cell(p, fs, lam)
        f_newton = bf.solve_implicit(fs, lam)
        np.testing.assert_allclose(f_closed, f_newton, rtol=1e-11, atol=1e-14)


def test_relaxation_gaussian_is_G_of_result(orc):
    """The Gaussian used by the closed form is G evaluated on the relaxed f."""
    p = grid(orc, nv=12, vmax=5.0)
    fs = np.random.default_rng(2).uniform(0.05, 1.0, p.nv2)
    f, g, _ = orc.relax_cell(p, fs, 0.8)
    np.testing.assert_allclose(orc.gaussian_of(p, f), g, rtol=1e-11, atol=1e-15)


def test_relaxation_stiff_limit_is_maxwellian(orc):
    """lam -> infinity: f -> Mhat(rho, u, T) (asymptotic preservation, Sec. 3.6)."""
    p = grid(orc, nv=12, vmax=5.0)
    fs = np.random.default_rng(4).uniform(0.05, 1.0, p.nv2)
    f, _, _ = orc.relax_cell(p, fs, 1e13)
    mo = orc.moments(p, fs)
    np.testing.assert_allclose(f, orc.maxwellian_hat(p, *mo[:4]), rtol=1e-10, atol=1e-13)


def test_l1_distance_matches_direct_sum(orc):
    p = grid(orc, nv=16, vmax=6.0)
    m1 = orc.maxwellian(p, 1.0, 0.5, 0.0, 1.0)
    m2 = orc.maxwellian(p, 0.7, -0.5, 0.2, 0.6)
    f = m1 + m2
    rho, ux, uy, T, _ = np_moments(p, f)
    vx, vy = orc.velocity_nodes(p)
    mref = rho * multivariate_normal(mean=[ux, uy], cov=T * np.eye(2)).pdf(np.c_[vx, vy])
    w = (2 * p.vmax / p.nv) ** 2
    assert abs(orc.l1_to_maxwellian(p, f) - w * np.abs(f - mref).sum()) < 1e-12
    assert orc.l1_to_maxwellian(p, orc.maxwellian(p, 1.0, 0.0, 0.0, 1.0)) < 1e-6
