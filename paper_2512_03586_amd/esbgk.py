"""Thin ctypes binding of libesbgk.so (include/esbgk.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (``torch.empty(..., device="cuda")``)
and the current HIP stream; nothing here computes on the host.  If the
library or a GPU is missing the calls raise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# ESBGK_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("ESBGK_LIB", os.path.join(_HERE, "libesbgk.so"))

OK, EINVAL, ENOMEM, EDEVICE, ENONPHYS = 0, -1, -2, -3, -4
ARS222, ARS233 = 0, 1
UPWIND1, MINMOD2 = 0, 1
FP64, FP32, BF16, MIXED = 0, 1, 2, 3
IND_PLAIN, IND_FROZEN, IND_LEARNED = 0, 1, 2
COUPLE_STAGE, COUPLE_STEP = 0, 1


class EsbgkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"esbgk error {code}: {msg}")
        self.code = code


class esbgk_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nv", C.c_int32),
                ("scheme", C.c_int32), ("recon", C.c_int32), ("precision", C.c_int32),
                ("indicator", C.c_int32), ("ce_set", C.c_int32), ("correction", C.c_int32),
                ("coupling", C.c_int32), ("learned_k", C.c_int32), ("reserved", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("vmax", C.c_double),
                ("beta", C.c_double), ("tau", C.c_double), ("cfl", C.c_double), ("dt", C.c_double),
                ("eta", C.c_double), ("delta", C.c_double)]


class esbgk_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("time", C.c_double), ("dt", C.c_double),
                ("n_kinetic", C.c_int32), ("n_buffer", C.c_int32), ("error_flags", C.c_int32),
                ("reserved", C.c_int32), ("kinetic_cell_steps", C.c_int64)]


K_STAGE2, K_STAGE3, K_FINAL, K_FILL, K_COUNT = 0, 1, 2, 3, 4


def make_config(nx, ny, nv, vmax, *, lx=1.0, ly=1.0, scheme=ARS233, recon=MINMOD2, precision=FP32,
                indicator=IND_PLAIN, ce_set=0, correction=1, coupling=COUPLE_STAGE, learned_k=10,
                beta=-0.5, tau=1.0, cfl=0.5, dt=0.0, eta=1e-2, delta=1e-3) -> esbgk_config:
    return esbgk_config(nx, ny, nv, scheme, recon, precision, indicator, ce_set, correction, coupling,
                        learned_k, 0, lx, ly, vmax, beta, tau, cfl, dt, eta, delta)


_lib = None
_VP = C.c_void_p


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_03586_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(esbgk_config)
        sig = {
            "esbgk_workspace_size": [P, C.POINTER(C.c_size_t)],
            "esbgk_create": [P, _VP, C.c_size_t, C.POINTER(_VP)],
            "esbgk_set_state": [_VP, _VP, _VP, _VP, _VP, _VP, _VP],
            "esbgk_set_mask": [_VP, _VP, _VP],
            "esbgk_set_f": [_VP, _VP, _VP],
            "esbgk_step": [_VP, C.c_int, _VP],
            "esbgk_get_moments": [_VP, _VP, _VP, _VP, _VP, _VP],
            "esbgk_get_conserved": [_VP, _VP, _VP],
            "esbgk_get_mask": [_VP, _VP, _VP],
            "esbgk_get_f": [_VP, _VP, _VP],
            "esbgk_get_l1": [_VP, _VP, _VP],
            "esbgk_get_kinetic_cells": [_VP, _VP, C.POINTER(C.c_int32), _VP],
            "esbgk_get_stats": [_VP, C.POINTER(esbgk_stats), _VP],
            "esbgk_indicator": [P, _VP, _VP, _VP, _VP, _VP, _VP, _VP],
            "esbgk_set_timing": [_VP, C.c_int],
            "esbgk_kernel_times": [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int],
            "esbgk_mlp_param_count": [],
            "esbgk_mlp_workspace_size": [C.c_int, C.POINTER(C.c_size_t)],
            "esbgk_mlp_create": [C.c_int, _VP, C.c_size_t, C.POINTER(_VP)],
            "esbgk_mlp_set_weights": [_VP, _VP, _VP],
            "esbgk_mlp_get_weights": [_VP, _VP, _VP],
            "esbgk_mlp_derived": [C.c_int, C.c_int, C.c_double, C.c_double, _VP, C.c_int, _VP, _VP],
            "esbgk_mlp_features": [C.c_int, C.c_int, _VP, _VP, C.c_int, _VP, C.c_int, _VP, _VP],
            "esbgk_mlp_forward": [_VP, _VP, C.c_int, _VP, _VP],
            "esbgk_mlp_gradients": [_VP, _VP, _VP, C.c_int, C.c_float, _VP, _VP, _VP],
            "esbgk_mlp_train_step": [_VP, _VP, _VP, C.c_int, C.c_float, C.c_float, _VP, _VP],
            "esbgk_set_learned": [_VP, _VP, C.c_float, C.c_int],
            "esbgk_get_learned_stats": [_VP, C.POINTER(C.c_int64), _VP],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.esbgk_destroy.argtypes = [_VP]
        L.esbgk_destroy.restype = None
        L.esbgk_last_error.argtypes = []
        L.esbgk_last_error.restype = C.c_char_p
        L.esbgk_mlp_destroy.argtypes = [_VP]
        L.esbgk_mlp_destroy.restype = None
        L.esbgk_mlp_last_error.argtypes = []
        L.esbgk_mlp_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != OK:
        raise EsbgkError(rc, lib().esbgk_last_error().decode())
    return rc


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- C entry points

def esbgk_workspace_size(cfg: esbgk_config) -> int:
    n = C.c_size_t(0)
    _check(lib().esbgk_workspace_size(C.byref(cfg), C.byref(n)))
    return n.value


def esbgk_create(cfg: esbgk_config, workspace: torch.Tensor) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(lib().esbgk_create(C.byref(cfg), _ptr(workspace), workspace.numel() * workspace.element_size(),
                              C.byref(ctx)))
    return ctx


def esbgk_destroy(ctx) -> None:
    lib().esbgk_destroy(ctx)


def esbgk_set_state(ctx, rho, ux, uy, T, eps, stream=None):
    return _check(lib().esbgk_set_state(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(eps), _stream(stream)))


def esbgk_set_mask(ctx, mask, stream=None):
    return _check(lib().esbgk_set_mask(ctx, _ptr(mask), _stream(stream)))


def esbgk_set_f(ctx, f, stream=None):
    return _check(lib().esbgk_set_f(ctx, _ptr(f), _stream(stream)))


def esbgk_step(ctx, nsteps: int, stream=None):
    return _check(lib().esbgk_step(ctx, int(nsteps), _stream(stream)))


def esbgk_get_moments(ctx, rho=None, ux=None, uy=None, T=None, stream=None):
    return _check(lib().esbgk_get_moments(ctx, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _stream(stream)))


def esbgk_get_conserved(ctx, U, stream=None):
    return _check(lib().esbgk_get_conserved(ctx, _ptr(U), _stream(stream)))


def esbgk_get_mask(ctx, mask, stream=None):
    return _check(lib().esbgk_get_mask(ctx, _ptr(mask), _stream(stream)))


def esbgk_get_f(ctx, f, stream=None):
    return _check(lib().esbgk_get_f(ctx, _ptr(f), _stream(stream)))


def esbgk_get_l1(ctx, l1, stream=None):
    return _check(lib().esbgk_get_l1(ctx, _ptr(l1), _stream(stream)))


def esbgk_get_kinetic_cells(ctx, cells, stream=None) -> int:
    n = C.c_int32(0)
    _check(lib().esbgk_get_kinetic_cells(ctx, _ptr(cells), C.byref(n), _stream(stream)))
    return n.value


def esbgk_get_stats(ctx, stream=None, check=True) -> esbgk_stats:
    s = esbgk_stats()
    rc = lib().esbgk_get_stats(ctx, C.byref(s), _stream(stream))
    if check:
        _check(rc)
    return s


def esbgk_indicator(cfg: esbgk_config, prim, eps, l1, mask_old, mask_new, lam=None, stream=None):
    return _check(lib().esbgk_indicator(C.byref(cfg), _ptr(prim), _ptr(eps), _ptr(l1), _ptr(mask_old),
                                        _ptr(mask_new), _ptr(lam), _stream(stream)))


def esbgk_set_timing(ctx, enable: bool):
    return _check(lib().esbgk_set_timing(ctx, int(bool(enable))))


def esbgk_kernel_times(ctx, reset: bool = True):
    """(milliseconds, launches) per kernel class K_STAGE2..K_FILL."""
    ms = (C.c_double * K_COUNT)()
    n = (C.c_int64 * K_COUNT)()
    _check(lib().esbgk_kernel_times(ctx, ms, n, int(bool(reset))))
    return list(ms), list(n)


def _mcheck(rc: int) -> int:
    if rc != OK:
        raise EsbgkError(rc, lib().esbgk_mlp_last_error().decode())
    return rc


def esbgk_mlp_param_count() -> int:
    return lib().esbgk_mlp_param_count()


def esbgk_mlp_workspace_size(max_batch: int) -> int:
    n = C.c_size_t(0)
    _mcheck(lib().esbgk_mlp_workspace_size(int(max_batch), C.byref(n)))
    return n.value


def esbgk_mlp_create(max_batch: int, workspace: torch.Tensor) -> C.c_void_p:
    net = C.c_void_p()
    _mcheck(lib().esbgk_mlp_create(int(max_batch), _ptr(workspace), workspace.numel(), C.byref(net)))
    return net


def esbgk_mlp_destroy(net):
    lib().esbgk_mlp_destroy(net)


def esbgk_mlp_set_weights(net, params, stream=None):
    return _mcheck(lib().esbgk_mlp_set_weights(net, _ptr(params), _stream(stream)))


def esbgk_mlp_get_weights(net, params, stream=None):
    return _mcheck(lib().esbgk_mlp_get_weights(net, _ptr(params), _stream(stream)))


def esbgk_mlp_derived(nx, ny, lx, ly, fields, nsnap, derived, stream=None):
    return _mcheck(lib().esbgk_mlp_derived(int(nx), int(ny), float(lx), float(ly), _ptr(fields), int(nsnap),
                                           _ptr(derived), _stream(stream)))


def esbgk_mlp_features(nx, ny, fields, derived, nsnap, samples, n, X, stream=None):
    return _mcheck(lib().esbgk_mlp_features(int(nx), int(ny), _ptr(fields), _ptr(derived), int(nsnap), _ptr(samples),
                                            int(n), _ptr(X), _stream(stream)))


def esbgk_mlp_forward(net, X, n, logits, stream=None):
    return _mcheck(lib().esbgk_mlp_forward(net, _ptr(X), int(n), _ptr(logits), _stream(stream)))


def esbgk_mlp_gradients(net, X, y, n, w_pos, grad, loss=None, stream=None):
    return _mcheck(lib().esbgk_mlp_gradients(net, _ptr(X), _ptr(y), int(n), float(w_pos), _ptr(grad), _ptr(loss),
                                             _stream(stream)))


def esbgk_mlp_train_step(net, X, y, n, w_pos, lr, loss=None, stream=None):
    return _mcheck(lib().esbgk_mlp_train_step(net, _ptr(X), _ptr(y), int(n), float(w_pos), float(lr), _ptr(loss),
                                              _stream(stream)))


def esbgk_set_learned(ctx, net, threshold: float, dilation: int = 0):
    return _check(lib().esbgk_set_learned(ctx, net, float(threshold), int(dilation)))


def esbgk_get_learned_stats(ctx, stream=None):
    """(checks, missed, extra, plain-kinetic cells) summed over check steps."""
    out = (C.c_int64 * 4)()
    _check(lib().esbgk_get_learned_stats(ctx, out, _stream(stream)))
    return tuple(out)


# ---------------------------------------------------------------- convenience

class Network:
    """The learned-indicator network plus its workspace."""

    def __init__(self, max_batch: int, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("esbgk needs a GPU (no CPU path exists)")
        self.max_batch = int(max_batch)
        self.nparam = esbgk_mlp_param_count()
        nbytes = esbgk_mlp_workspace_size(max_batch)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.net = esbgk_mlp_create(max_batch, self._ws)
        self.device = device
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)

    def __del__(self):
        try:
            if getattr(self, "net", None) is not None:
                esbgk_mlp_destroy(self.net)
                self.net = None
        except Exception:
            pass

    def set_weights(self, params):
        esbgk_mlp_set_weights(self.net, torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous())

    def get_weights(self):
        out = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        esbgk_mlp_get_weights(self.net, out)
        return out

    def forward(self, X):
        z = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        esbgk_mlp_forward(self.net, X, X.shape[0], z)
        return z

    def gradients(self, X, y, w_pos):
        g = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        esbgk_mlp_gradients(self.net, X, y, X.shape[0], w_pos, g, self.loss)
        return g, self.loss

    def train_step(self, X, y, w_pos, lr):
        esbgk_mlp_train_step(self.net, X, y, X.shape[0], w_pos, lr, self.loss)
        return self.loss


def mlp_features(nx, ny, lx, ly, fields, samples):
    """BF16 feature rows (as int16 bit patterns, [n][192]) of samples (int32
    [n][2] = snapshot, cell) of the snapshot fields (FP64 [nsnap][6][nc])."""
    nsnap = fields.shape[0]
    derived = torch.empty(nsnap, 3, nx * ny, dtype=torch.float64, device=fields.device)
    esbgk_mlp_derived(nx, ny, lx, ly, fields, nsnap, derived)
    X = torch.empty(samples.shape[0], 192, dtype=torch.int16, device=fields.device)
    esbgk_mlp_features(nx, ny, fields, derived, nsnap, samples, samples.shape[0], X)
    return X


class Engine:
    """A context plus its workspace (a torch uint8 device tensor)."""

    def __init__(self, cfg: esbgk_config, device: str = "cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("esbgk needs a GPU (no CPU path exists)")
        self.cfg = cfg
        self.nc = cfg.nx * cfg.ny
        self.nv2 = cfg.nv * cfg.nv
        nbytes = esbgk_workspace_size(cfg)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:off + nbytes]
        self.ctx = esbgk_create(cfg, self._ws)
        self.device = device

    def __del__(self):
        try:
            if getattr(self, "ctx", None) is not None:
                esbgk_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def _dev(self, a, dtype=torch.float64):
        return torch.as_tensor(a, dtype=dtype).to(self.device).contiguous()

    def set_state(self, rho, ux, uy, T, eps):
        esbgk_set_state(self.ctx, *(self._dev(a) for a in (rho, ux, uy, T, eps)))

    def set_mask(self, mask):
        esbgk_set_mask(self.ctx, self._dev(mask, torch.uint8))

    def set_f(self, f):
        esbgk_set_f(self.ctx, self._dev(f).reshape(-1))

    def step(self, n=1):
        esbgk_step(self.ctx, n)

    def moments(self):
        out = [torch.empty(self.nc, dtype=torch.float64, device=self.device) for _ in range(4)]
        esbgk_get_moments(self.ctx, *out)
        return out

    def conserved(self):
        U = torch.empty(4, self.nc, dtype=torch.float64, device=self.device)
        esbgk_get_conserved(self.ctx, U)
        return U

    def mask(self):
        m = torch.empty(self.nc, dtype=torch.uint8, device=self.device)
        esbgk_get_mask(self.ctx, m)
        return m

    def f(self):
        f = torch.empty(self.nc, self.nv2, dtype=torch.float64, device=self.device)
        esbgk_get_f(self.ctx, f)
        return f

    def l1(self):
        l1 = torch.empty(self.nc, dtype=torch.float64, device=self.device)
        esbgk_get_l1(self.ctx, l1)
        return l1

    def kinetic_cells(self):
        cells = torch.empty(self.nc, dtype=torch.int32, device=self.device)
        n = esbgk_get_kinetic_cells(self.ctx, cells)
        return cells[:n]

    def stats(self, check=True):
        return esbgk_get_stats(self.ctx, check=check)

    def set_learned(self, network=None, threshold=0.0, dilation=0):
        self._network = network   # keep it alive while attached
        esbgk_set_learned(self.ctx, network.net if network is not None else None, threshold, dilation)

    def learned_stats(self):
        return esbgk_get_learned_stats(self.ctx)
