"""TEST INFRASTRUCTURE, NOT PRODUCT CODE: FP64 NumPy oracle of the learned
regime indicator (features, MLP forward/backward, loss, Adam).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module; the GPU path shares no code with it.

The learned indicator replaces the plain criterion of Sec. 3.1.2 between
checks: from the macroscopic state at the start of a step it predicts which
cells the plain criterion will mark kinetic at any of the next K steps.  The
paper has no learned component; everything here follows the definitions
below, which the GPU kernels implement independently.

Features of cell c (periodic 5 x 5 stencil, offsets dj = -2..2 outer,
di = -2..2 inner, stencil index k = 5 (dj + 2) + (di + 2)); for stencil cell s:
    f[7k + 0] = rho_s / rho_c - 1
    f[7k + 1] = ux_s - ux_c
    f[7k + 2] = uy_s - uy_c
    f[7k + 3] = T_s / T_c - 1
    f[7k + 4] = eps_s / (eps_s + 0.01)
    f[7k + 5] = A_s / (A_s + 1e-4),  A = eps^2 |grad u|^2
    f[7k + 6] = B_s / (B_s + 1e-4),  B = eps^2 |grad T|^2 / T
    f[175]    = previous mask of c (1 kinetic, 0 fluid);  f[176..191] = 0,
with central differences (q_{i+1} - q_{i-1}) / (2 dx) and
|grad u|^2 = ((ux_x^2 + ux_y^2) + uy_x^2) + uy_y^2.  A and B are the scales of
the two terms of S1 - I (the velocity-gradient and heat-flux terms), squashed
into [0, 1) by rational functions.  Every feature is a fixed sequence of
correctly rounded FP64 + - * /, then rounded to FP32 (nearest even) and to
BF16 (nearest even).

Network: z = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3 with x in R^192,
64 and 64 hidden units; the weights W1, W2, w3 enter rounded to BF16, the
biases in FP32; the hidden activations are stored rounded to BF16 (both are
inputs of the next product).  Loss: mean weighted logistic loss
    l = w_pos y softplus(-z) + (1 - y) softplus(z).
The gradients are those of the loss with respect to the rounded weights
(used for the FP32 master weights).  Adam: Kingma & Ba (2015), bias-corrected.
"""
from __future__ import annotations

import numpy as np

NFEAT, NIN, NH = 176, 192, 64
EPS_SCALE, GRAD_SCALE = 0.01, 1e-4


# ------------------------------------------------------------ rounding

def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_round(x):
    """FP64 -> FP32 (nearest even) -> BF16 (nearest even), returned as FP64."""
    f = to_f32(x)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    """BF16 bit patterns (uint16) of bf16_round(x)."""
    return (to_f32(bf16_round(x)).view(np.uint32) >> 16).astype(np.uint16)


# ------------------------------------------------------------ features

def _cd(q, nx, ny, dx, dy):
    Q = q.reshape(ny, nx)
    gx = (np.roll(Q, -1, axis=1) - np.roll(Q, 1, axis=1)) / (2.0 * dx)
    gy = (np.roll(Q, -1, axis=0) - np.roll(Q, 1, axis=0)) / (2.0 * dy)
    return gx.ravel(), gy.ravel()


def derived_fields(nx, ny, lx, ly, rho, ux, uy, T, eps):
    """Per-cell e, gA, gB of the feature definition (FP64, no contraction)."""
    dx, dy = lx / nx, ly / ny
    uxx, uxy = _cd(ux, nx, ny, dx, dy)
    uyx, uyy = _cd(uy, nx, ny, dx, dy)
    Tx, Ty = _cd(T, nx, ny, dx, dy)
    gu2 = ((uxx * uxx + uxy * uxy) + uyx * uyx) + uyy * uyy
    gT2 = Tx * Tx + Ty * Ty
    e2 = eps * eps
    A = e2 * gu2
    B = (e2 * gT2) / T
    return eps / (eps + EPS_SCALE), A / (A + GRAD_SCALE), B / (B + GRAD_SCALE)


def features(nx, ny, lx, ly, rho, ux, uy, T, eps, mask_prev, cells=None):
    """Feature rows (n x 192, FP64 values of BF16 numbers) of the given cells
    (default: all, row-major c = i + nx j)."""
    e, gA, gB = derived_fields(nx, ny, lx, ly, rho, ux, uy, T, eps)
    cells = np.arange(nx * ny) if cells is None else np.asarray(cells)
    i, j = cells % nx, cells // nx
    X = np.zeros((len(cells), NIN))
    for dj in range(-2, 3):
        for di in range(-2, 3):
            k = 5 * (dj + 2) + (di + 2)
            s = ((j + dj) % ny) * nx + (i + di) % nx
            X[:, 7 * k + 0] = rho[s] / rho[cells] - 1.0
            X[:, 7 * k + 1] = ux[s] - ux[cells]
            X[:, 7 * k + 2] = uy[s] - uy[cells]
            X[:, 7 * k + 3] = T[s] / T[cells] - 1.0
            X[:, 7 * k + 4] = e[s]
            X[:, 7 * k + 5] = gA[s]
            X[:, 7 * k + 6] = gB[s]
    X[:, 175] = mask_prev[cells].astype(np.float64)
    return bf16_round(X)


# ------------------------------------------------------------ network

def init_params(seed=0):
    """He-uniform initial weights (FP32 values), zero biases."""
    rng = np.random.default_rng(seed)
    def he(fan_in, shape):
        b = np.sqrt(6.0 / fan_in)
        return to_f32(rng.uniform(-b, b, size=shape)).astype(np.float64)
    W1 = he(NFEAT, (NIN, NH))
    W1[NFEAT:] = 0.0
    return dict(W1=W1, b1=np.zeros(NH), W2=he(NH, (NH, NH)), b2=np.zeros(NH),
                w3=he(NH, (NH,)), b3=np.zeros(()))


def forward(p, X, rounded=True):
    """Returns (z, cache).  rounded=False drops every BF16 rounding (a smooth
    function, for finite-difference checks)."""
    r = bf16_round if rounded else (lambda a: a)
    W1, W2, w3 = r(p["W1"]), r(p["W2"]), r(p["w3"])
    Z1 = X @ W1 + p["b1"]
    H1 = r(np.maximum(Z1, 0.0))
    Z2 = H1 @ W2 + p["b2"]
    H2 = r(np.maximum(Z2, 0.0))
    z = H2 @ w3 + p["b3"]
    return z, dict(X=X, W1=W1, W2=W2, w3=w3, H1=H1, H2=H2)


def softplus(x):
    return np.log1p(np.exp(-np.abs(x))) + np.maximum(x, 0.0)


def loss(z, y, wpos):
    return float(np.mean(wpos * y * softplus(-z) + (1.0 - y) * softplus(z)))


def backward(z, y, wpos, cache):
    """Gradients of the mean weighted logistic loss; ReLU'(0) = 0."""
    n = z.shape[0]
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (sig * (wpos * y + 1.0 - y) - wpos * y) / n
    H1, H2, X = cache["H1"], cache["H2"], cache["X"]
    g = {"w3": H2.T @ dz, "b3": np.asarray(dz.sum())}
    dZ2 = np.outer(dz, cache["w3"]) * (H2 > 0.0)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ cache["W2"].T) * (H1 > 0.0)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def loss_and_grads(p, X, y, wpos, rounded=True):
    z, cache = forward(p, X, rounded)
    return loss(z, y, wpos), backward(z, y, wpos, cache)


ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def flatten(p):
    """Flat parameter vector in the ABI's order: W1 (192 x 64, row-major by
    input), b1, W2 (64 x 64), b2, w3, b3."""
    return np.concatenate([np.ravel(p[k]) for k in ORDER])


def unflatten(v):
    shapes = dict(W1=(NIN, NH), b1=(NH,), W2=(NH, NH), b2=(NH,), w3=(NH,), b3=())
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(shapes[k])) if shapes[k] else 1
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shapes[k])
        o += n
    return out


NPARAM = NIN * NH + NH + NH * NH + NH + NH + 1


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t >= 1) on flat vectors; returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
