"""FP64 CPU oracle of the coupled IMEX ES-BGK scheme -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_2512_03586_amd``)
never does, and the two share no code: this wrapper loads ``liboracle.so``,
built from ``esbgk_oracle.c`` by :func:`build` with gcc (``-O2 -fopenmp
-ffp-contract=off``, no fast-math).

Every function forwards to the C routine of the same name; the C source cites
the passage of arXiv 2512.03586 each routine follows.  Arrays are numpy
float64 / uint8, C-contiguous.  Layouts: ``f`` is ``[nc, nv*nv]`` (cell
``i + nx*j``, node ``a + nv*b``), ``U`` and ``prim`` are SoA ``[4, nc]``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esbgk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so next to its source (gcc, FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Cfg(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nv", C.c_int32),
                ("scheme", C.c_int32), ("recon", C.c_int32), ("correction", C.c_int32),
                ("ce_set", C.c_int32), ("coupling", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("vmax", C.c_double),
                ("beta", C.c_double), ("tau", C.c_double), ("dt", C.c_double),
                ("eta", C.c_double), ("delta", C.c_double)]


@dataclass
class Problem:
    """Parameters of one run (names follow the paper's notation)."""
    nx: int
    ny: int
    nv: int
    vmax: float
    lx: float = 1.0
    ly: float = 1.0
    scheme: int = 1          # 0 = ARS(2,2,2), 1 = ARS(2,3,3)
    recon: int = 1           # 0 = first-order upwind, 1 = minmod
    correction: int = 1      # 1 = six-moment discrete-conservation correction
    ce_set: int = 0          # 0 = paper constants, 1 = 2D-consistent
    coupling: int = 0        # 0 = every stage (Algorithm 1), 1 = once per step (LOC)
    beta: float = -0.5
    tau: float = 1.0
    dt: float = 0.0          # 0 -> cfl * min(dx, dy) / vmax
    cfl: float = 0.5
    eta: float = 1e-2
    delta: float = 1e-3

    def cfg(self) -> Cfg:
        dt = self.dt if self.dt > 0 else self.cfl * min(self.lx / self.nx, self.ly / self.ny) / self.vmax
        return Cfg(self.nx, self.ny, self.nv, self.scheme, self.recon, self.correction,
                   self.ce_set, self.coupling, self.lx, self.ly, self.vmax, self.beta,
                   self.tau, dt, self.eta, self.delta)

    @property
    def nc(self) -> int:
        return self.nx * self.ny

    @property
    def nv2(self) -> int:
        return self.nv * self.nv


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        P = C.POINTER(Cfg)
        d = C.POINTER(C.c_double)
        u8 = C.POINTER(C.c_uint8)
        sig = {
            "orc_velocity_nodes": (None, [P, d, d]),
            "orc_tableau": (None, [C.c_int, d, d, d, d]),
            "orc_moments": (None, [P, d, d]),
            "orc_maxwellian": (None, [P, C.c_double, C.c_double, C.c_double, C.c_double, d]),
            "orc_gaussian_tilde": (C.c_int, [P] + [C.c_double] * 6 + [d]),
            "orc_gaussian_hat": (C.c_int, [P] + [C.c_double] * 7 + [d, d]),
            "orc_maxwellian_hat": (C.c_int, [P] + [C.c_double] * 4 + [d]),
            "orc_gaussian_of": (C.c_int, [P, d, d]),
            "orc_relax_cell": (C.c_int, [P, d, C.c_double, d, d, d]),
            "orc_transport": (None, [P, d, d]),
            "orc_euler_phi": (None, [P, d, d]),
            "orc_l1_to_maxwellian": (C.c_double, [P, d]),
            "orc_indicator": (None, [P, d, d, d, u8, u8, d]),
            "orc_primitives": (None, [C.c_size_t, d, d]),
            "orc_regime_update": (C.c_int, [P, d, d, d, u8, d]),
            "orc_step_once": (C.c_int, [P, d, d, u8, d]),
            "orc_run": (C.c_int, [P, d, d, u8, d, d, C.c_int, C.c_int]),
            "orc_euler_flux": (None, [d, C.c_int, d]),
            "orc_rusanov": (None, [d, d, C.c_int, d]),
            "orc_num_threads": (C.c_int, []),
            "orc_set_num_threads": (None, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u8(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_uint8))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- wrappers

def velocity_nodes(p: Problem):
    vx = np.empty(p.nv2); vy = np.empty(p.nv2)
    lib().orc_velocity_nodes(C.byref(p.cfg()), _d(vx), _d(vy))
    return vx, vy


def tableau(scheme: int):
    At = np.empty(9); bt = np.empty(3); A = np.empty(9); b = np.empty(3)
    lib().orc_tableau(scheme, _d(At), _d(bt), _d(A), _d(b))
    return At.reshape(3, 3), bt, A.reshape(3, 3), b


def moments(p: Problem, fc) -> np.ndarray:
    """{rho, ux, uy, T, Thxx, Thxy, Thyy} of one cell."""
    fc = _f64(fc); out = np.empty(7)
    lib().orc_moments(C.byref(p.cfg()), _d(fc), _d(out))
    return out


def maxwellian(p: Problem, rho, ux, uy, T) -> np.ndarray:
    m = np.empty(p.nv2)
    lib().orc_maxwellian(C.byref(p.cfg()), rho, ux, uy, T, _d(m))
    return m


def gaussian_tilde(p: Problem, rho, ux, uy, txx, txy, tyy) -> np.ndarray:
    g = np.empty(p.nv2)
    rc = lib().orc_gaussian_tilde(C.byref(p.cfg()), rho, ux, uy, txx, txy, tyy, _d(g))
    if rc:
        raise ValueError("tensor not positive definite")
    return g


def gaussian_hat(p: Problem, rho, ux, uy, T, txx, txy, tyy, return_coef=False):
    g = np.empty(p.nv2); c = np.empty(6)
    rc = lib().orc_gaussian_hat(C.byref(p.cfg()), rho, ux, uy, T, txx, txy, tyy, _d(g), _d(c))
    if rc:
        raise ValueError(f"gaussian_hat failed ({rc})")
    return (g, c) if return_coef else g


def maxwellian_hat(p: Problem, rho, ux, uy, T) -> np.ndarray:
    m = np.empty(p.nv2)
    rc = lib().orc_maxwellian_hat(C.byref(p.cfg()), rho, ux, uy, T, _d(m))
    if rc:
        raise ValueError("maxwellian_hat failed")
    return m


def gaussian_of(p: Problem, fc) -> np.ndarray:
    fc = _f64(fc); g = np.empty(p.nv2)
    if lib().orc_gaussian_of(C.byref(p.cfg()), _d(fc), _d(g)):
        raise ValueError("gaussian_of failed")
    return g


def relax_cell(p: Problem, fstar, lam):
    """Closed-form implicit stage; returns (f, G, {rho,ux,uy,T,txx,txy,tyy})."""
    fstar = _f64(fstar); f = np.empty(p.nv2); g = np.empty(p.nv2); mo = np.empty(7)
    if lib().orc_relax_cell(C.byref(p.cfg()), _d(fstar), float(lam), _d(f), _d(g), _d(mo)):
        raise ValueError("relax failed")
    return f, g, mo


def transport(p: Problem, f) -> np.ndarray:
    f = _f64(f).reshape(p.nc, p.nv2); out = np.empty_like(f)
    lib().orc_transport(C.byref(p.cfg()), _d(f), _d(out))
    return out


def euler_phi(p: Problem, U) -> np.ndarray:
    U = _f64(U).reshape(4, p.nc); out = np.empty_like(U)
    lib().orc_euler_phi(C.byref(p.cfg()), _d(U), _d(out))
    return out


def euler_flux(U4, d: int) -> np.ndarray:
    """Physical Euler flux of one state U = (rho, mx, my, E) in direction d."""
    U4 = _f64(U4); out = np.empty(4)
    lib().orc_euler_flux(_d(U4), int(d), _d(out))
    return out


def rusanov(UL, UR, d: int) -> np.ndarray:
    UL = _f64(UL); UR = _f64(UR); out = np.empty(4)
    lib().orc_rusanov(_d(UL), _d(UR), int(d), _d(out))
    return out


def l1_to_maxwellian(p: Problem, fc) -> float:
    fc = _f64(fc)
    return lib().orc_l1_to_maxwellian(C.byref(p.cfg()), _d(fc))


def indicator(p: Problem, prim, eps, l1, mask_old, return_lambda=False):
    prim = _f64(prim).reshape(4, p.nc); eps = _f64(eps); l1 = _f64(l1)
    mo = np.ascontiguousarray(mask_old, dtype=np.uint8)
    mn = np.empty(p.nc, np.uint8); lam = np.empty(p.nc)
    lib().orc_indicator(C.byref(p.cfg()), _d(prim), _d(eps), _d(l1), _u8(mo), _u8(mn), _d(lam))
    return (mn, lam) if return_lambda else mn


def primitives(U) -> np.ndarray:
    U = _f64(U); nc = U.shape[-1]; out = np.empty((4, nc))
    lib().orc_primitives(nc, _d(U), _d(out))
    return out


def conserved(rho, ux, uy, T) -> np.ndarray:
    rho = np.asarray(rho, np.float64); ux = np.asarray(ux, np.float64)
    uy = np.asarray(uy, np.float64); T = np.asarray(T, np.float64)
    return np.ascontiguousarray(np.stack([rho, rho * ux, rho * uy,
                                          0.5 * rho * (ux * ux + uy * uy) + rho * T]))


class State:
    """Oracle state: f [nc, nv2], U [4, nc], mask [nc], eps [nc], l1 [nc]."""

    def __init__(self, p: Problem, U, eps, f=None, mask=None):
        self.p = p
        self.U = _f64(U).reshape(4, p.nc).copy()
        self.eps = _f64(eps).reshape(p.nc).copy()
        self.f = np.zeros((p.nc, p.nv2)) if f is None else _f64(f).reshape(p.nc, p.nv2).copy()
        self.mask = np.zeros(p.nc, np.uint8) if mask is None else \
            np.ascontiguousarray(mask, dtype=np.uint8).reshape(p.nc).copy()
        self.l1 = np.zeros(p.nc)

    @classmethod
    def from_primitives(cls, p: Problem, rho, ux, uy, T, eps, mask=None):
        """U from (rho, u, T); kinetic cells (mask = 1) get f = Mhat(U)."""
        U = conserved(rho, ux, uy, T)
        st = cls(p, U, eps, mask=mask)
        prim = primitives(st.U)
        for q in np.nonzero(st.mask)[0]:
            st.f[q] = maxwellian_hat(p, *prim[:, q])
        return st

    def run(self, nsteps: int, update_regime: bool = True) -> None:
        rc = lib().orc_run(C.byref(self.p.cfg()), _d(self.f), _d(self.U), _u8(self.mask),
                           _d(self.eps), _d(self.l1), int(nsteps), int(bool(update_regime)))
        if rc:
            raise FloatingPointError(f"oracle run failed ({rc})")

    def prim(self) -> np.ndarray:
        return primitives(self.U)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))
