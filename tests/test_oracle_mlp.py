"""Pins of the learned-indicator oracle (oracle/mlp.py): rounding against
torch's float32 -> bfloat16 conversion, the backward pass against finite
differences of the unrounded network, ReLU'(0) = 0, the loss and Adam against
torch's library routines, and the features against closed forms."""
import numpy as np
import pytest
import torch

from oracle import mlp as M


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -(1.0 + 2.0 ** -8), 65504.0,
                         1e-38, 3.4e38]])
    ref = torch.tensor(x, dtype=torch.float64).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16_round(x), ref)
    # ties go to even
    assert M.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert M.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    bits = M.bf16_bits(np.array([1.0, -2.0]))
    assert bits.tolist() == [0x3F80, 0xC000]


def _rand_problem(n=37, seed=1):
    rng = np.random.default_rng(seed)
    p = M.init_params(seed)
    for k in ("b1", "b2"):
        p[k] = rng.uniform(-0.1, 0.1, size=p[k].shape)
    p["b3"] = np.asarray(0.05)
    X = np.zeros((n, M.NIN))
    X[:, :M.NFEAT] = rng.uniform(-1, 1, size=(n, M.NFEAT))
    y = (rng.uniform(size=n) < 0.3).astype(np.float64)
    return p, X, y


def test_backward_matches_finite_differences_of_unrounded_network():
    p, X, y = _rand_problem()
    wpos = 3.0
    _, g = M.loss_and_grads(p, X, y, wpos, rounded=False)
    rng = np.random.default_rng(2)
    h = 1e-6
    for k in M.ORDER:
        idxs = [()] if p[k].ndim == 0 else [tuple(rng.integers(0, s) for s in p[k].shape) for _ in range(12)]
        if k == "W1":
            idxs = [(int(rng.integers(0, M.NFEAT)), int(rng.integers(0, M.NH))) for _ in range(12)]
        for ix in idxs:
            q = {a: b.copy() for a, b in p.items()}
            q[k] = np.array(q[k], dtype=np.float64)
            q[k][ix] += h
            lp = M.loss(M.forward(q, X, rounded=False)[0], y, wpos)
            q[k][ix] -= 2 * h
            lm = M.loss(M.forward(q, X, rounded=False)[0], y, wpos)
            fd = (lp - lm) / (2 * h)
            an = g[k][ix]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (k, ix, fd, an)


def test_relu_derivative_at_zero_is_zero():
    p, X, y = _rand_problem()
    p["W1"][:] = 0.0
    p["b1"][:] = 0.0          # every first-layer pre-activation is exactly 0
    _, g = M.loss_and_grads(p, X, y, 2.0)
    assert np.all(g["W1"] == 0.0) and np.all(g["b1"] == 0.0)
    assert np.all(g["W2"] == 0.0)
    assert np.any(g["b2"] != 0.0)


def test_loss_matches_torch_weighted_logistic_loss():
    rng = np.random.default_rng(3)
    z = rng.standard_normal(500) * 5
    y = (rng.uniform(size=500) < 0.4).astype(np.float64)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(
        torch.tensor(z), torch.tensor(y), pos_weight=torch.tensor(4.0)).item()
    assert abs(M.loss(z, y, 4.0) - ref) <= 1e-13 * abs(ref)


def test_gradient_of_logit_matches_torch_autograd():
    p, X, y = _rand_problem(n=50, seed=4)
    z = M.forward(p, X, rounded=False)[0]
    zt = torch.tensor(z, requires_grad=True)
    torch.nn.functional.binary_cross_entropy_with_logits(zt, torch.tensor(y), pos_weight=torch.tensor(2.5)).backward()
    _, g = M.loss_and_grads(p, X, y, 2.5, rounded=False)
    np.testing.assert_allclose(g["b3"], zt.grad.numpy().sum(), rtol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    w0 = rng.standard_normal(40)
    grads = [rng.standard_normal(40) for _ in range(4)]
    t = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(40), np.zeros(40)
    for s, gr in enumerate(grads, start=1):
        opt.zero_grad()
        t.grad = torch.tensor(gr)
        opt.step()
        w, m, v = M.adam(w, gr, m, v, s, 1e-2)
    np.testing.assert_allclose(w, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_flatten_roundtrip_and_size():
    p = M.init_params(7)
    v = M.flatten(p)
    assert v.size == M.NPARAM == 192 * 64 + 64 + 64 * 64 + 64 + 64 + 1
    q = M.unflatten(v)
    for k in M.ORDER:
        np.testing.assert_array_equal(q[k], p[k])
    assert np.all(p["W1"][M.NFEAT:] == 0.0)


# ------------------------------------------------------------ features

def _state(nx, ny, **kw):
    nc = nx * ny
    s = dict(rho=np.ones(nc), ux=np.zeros(nc), uy=np.zeros(nc), T=np.ones(nc), eps=np.full(nc, 1e-3),
             mask=np.zeros(nc, np.uint8))
    s.update(kw)
    return s


def _feat(nx, ny, s, lx=1.0, ly=1.0, cells=None):
    return M.features(nx, ny, lx, ly, s["rho"], s["ux"], s["uy"], s["T"], s["eps"], s["mask"], cells)


def test_features_of_uniform_state():
    nx, ny = 7, 6
    s = _state(nx, ny, mask=(np.arange(42) % 3 == 0).astype(np.uint8))
    X = _feat(nx, ny, s)
    for k in range(25):
        for m in (0, 1, 2, 3, 5, 6):
            assert np.all(X[:, 7 * k + m] == 0.0)
        assert np.all(X[:, 7 * k + 4] == M.bf16_round(1e-3 / (1e-3 + 0.01)))
    np.testing.assert_array_equal(X[:, 175], s["mask"])
    assert np.all(X[:, 176:] == 0.0)


def test_feature_stencil_order_and_periodic_wrap():
    nx, ny = 6, 5
    rho = np.ones(30)
    s0 = 0 * nx + 5                      # cell (i=5, j=0): at offset (+1, -1) of (0, 1) across both wraps
    rho[s0] = 2.0
    X = _feat(nx, ny, _state(nx, ny, rho=rho))
    c = 1 * nx + 0                       # centre (i=0, j=1)
    k = 5 * (-1 + 2) + (-1 + 2)          # (di, dj) = (-1, -1): i = -1 -> 5, j = 0
    row = X[c]
    assert row[7 * k] == 1.0
    others = [7 * q for q in range(25) if q != k]
    assert np.all(row[others] == 0.0)
    # the spike cell itself sees all its neighbours at -1/2
    assert X[s0, 7 * 12] == 0.0 and np.all(X[s0, [7 * q for q in range(25) if q != 12]] == -0.5)


def test_gradient_features_are_exact_for_linear_data_in_the_interior():
    nx, ny = 12, 12
    j = np.arange(144) // nx
    i = np.arange(144) % nx
    a, b = 0.3, 0.7
    ux = a * (j + 0.5) / ny               # linear in y, dy = 1/12
    T = 1.0 + b * (i + 0.5) / nx
    eps = np.full(144, 2e-2)
    X = _feat(nx, ny, _state(nx, ny, ux=ux, T=T, eps=eps))
    interior = [c for c in range(144) if 3 <= c % nx <= 8 and 3 <= c // nx <= 8]
    for c in interior:
        A = (2e-2 ** 2) * (a * a)
        gA = M.bf16_round(A / (A + 1e-4))
        assert abs(X[c, 7 * 12 + 5] - gA) <= 2.0 ** -8 * gA
        B = (2e-2 ** 2) * (b * b) / T[c]
        gB = M.bf16_round(B / (B + 1e-4))
        assert abs(X[c, 7 * 12 + 6] - gB) <= 2.0 ** -8 * gB


def test_features_for_a_subset_of_cells_equal_the_full_rows():
    nx, ny = 9, 8
    rng = np.random.default_rng(8)
    s = _state(nx, ny, rho=1 + 0.2 * rng.uniform(size=72), ux=rng.uniform(-1, 1, 72), uy=rng.uniform(-1, 1, 72),
               T=1 + 0.3 * rng.uniform(size=72), eps=10 ** rng.uniform(-4, 0, 72),
               mask=(rng.uniform(size=72) < 0.5).astype(np.uint8))
    full = _feat(nx, ny, s)
    cells = np.array([0, 8, 17, 71, 40])
    np.testing.assert_array_equal(_feat(nx, ny, s, cells=cells), full[cells])
    assert np.all(np.abs(full) <= 2.0)
