"""Training and evaluation of the learned regime indicator, on the GPU, with the
engine's own kernels (features, BF16 MFMA forward and backward, Adam).

Data: runs of the engine with the plain criterion (Sec. 3.1.2) on the
four-quadrant Riemann generator.  At every check step n (n a multiple of K)
a snapshot keeps the state at the start of the step, (rho, u, T, eps) and the
mask in use; its label marks the cells the plain criterion makes kinetic at
any of the steps n .. n+K-1.  The network is trained on random cells of
these snapshots with a weighted logistic loss (positives weighted w_pos), and
its threshold is set on held-out runs so that at most a fraction `miss` of
the positive cells falls below it.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import esbgk as E
from . import inputs


@dataclass
class Snapshots:
    nx: int
    ny: int
    lx: float
    ly: float
    fields: torch.Tensor      # FP64 [nsnap][6][nc]
    labels: torch.Tensor      # uint8 [nsnap][nc]
    derived: torch.Tensor = None

    @property
    def nsnap(self):
        return self.fields.shape[0]

    def prepare(self):
        self.derived = torch.empty(self.nsnap, 3, self.nx * self.ny, dtype=torch.float64, device=self.fields.device)
        E.esbgk_mlp_derived(self.nx, self.ny, self.lx, self.ly, self.fields, self.nsnap, self.derived)
        return self

    def features(self, samples):
        X = torch.empty(samples.shape[0], 192, dtype=torch.int16, device=self.fields.device)
        E.esbgk_mlp_features(self.nx, self.ny, self.fields, self.derived, self.nsnap, samples, samples.shape[0], X)
        return X


def plain_run_snapshots(seed, *, nx=256, nv=32, vmax=10.0, steps=200, K=10, precision=E.FP32, **gen):
    """Snapshots and labels of one plain-criterion run (config-2 generator)."""
    d = inputs.riemann4(nx=nx, ny=nx, nv=nv, vmax=vmax, seed=seed, **gen)
    cfg = E.make_config(nx, nx, nv, vmax, precision=precision, indicator=E.IND_PLAIN, scheme=E.ARS233,
                        recon=E.MINMOD2, eta=1e-2, delta=1e-3)
    eng = E.Engine(cfg)
    eng.set_state(d["rho"], d["ux"], d["uy"], d["T"], d["eps"])
    eps = torch.as_tensor(d["eps"], dtype=torch.float64, device="cuda")
    nc = nx * nx
    snaps, masks = [], []
    for n in range(steps):
        if n % K == 0:
            prim = torch.stack(eng.moments())
            mprev = eng.mask().to(torch.float64)
            snaps.append(torch.cat([prim, eps[None], mprev[None]], 0))
        eng.step(1)
        masks.append(eng.mask())
    M = torch.stack(masks)
    nwin = steps // K
    labels = torch.stack([M[w * K:(w + 1) * K].amax(0) for w in range(nwin)])
    return torch.stack(snaps[:nwin]), labels


def collect(seeds, **kw):
    F, Y = [], []
    nx = kw.get("nx", 256)
    for s in seeds:
        f, y = plain_run_snapshots(s, **kw)
        F.append(f)
        Y.append(y)
    return Snapshots(nx, nx, 1.0, 1.0, torch.cat(F), torch.cat(Y)).prepare()


@dataclass
class TrainResult:
    params: torch.Tensor
    threshold: float
    losses: list = field(default_factory=list)
    seconds: float = 0.0
    val_recall: float = 0.0
    val_positive_rate: float = 0.0
    val_predicted_rate: float = 0.0


def initial_params(seed=0):
    """He-uniform weights, zero biases (the flat ABI order)."""
    g = torch.Generator().manual_seed(seed)
    def he(fan_in, *shape):
        b = math.sqrt(6.0 / fan_in)
        return (torch.rand(*shape, generator=g, dtype=torch.float64) * 2 - 1) * b
    W1 = he(176, 192, 64)
    W1[176:] = 0
    parts = [W1.ravel(), torch.zeros(64), he(64, 64, 64).ravel(), torch.zeros(64), he(64, 64), torch.zeros(1)]
    return torch.cat([p.to(torch.float64) for p in parts]).to(torch.float32)


def random_samples(snaps: Snapshots, n, gen):
    nc = snaps.nx * snaps.ny
    s = torch.randint(0, snaps.nsnap, (n,), generator=gen, device="cpu")
    c = torch.randint(0, nc, (n,), generator=gen, device="cpu")
    return torch.stack([s, c], 1).to(torch.int32).cuda().contiguous()


def logits_of(net: E.Network, snaps: Snapshots, chunk=1 << 18):
    nc = snaps.nx * snaps.ny
    out = torch.empty(snaps.nsnap, nc, dtype=torch.float32, device="cuda")
    cells = torch.arange(nc, dtype=torch.int32, device="cuda")
    for k in range(snaps.nsnap):
        for a in range(0, nc, chunk):
            b = min(nc, a + chunk)
            smp = torch.stack([torch.full((b - a,), k, dtype=torch.int32, device="cuda"), cells[a:b]], 1).contiguous()
            out[k, a:b] = net.forward(snaps.features(smp))
    return out


def train(train_snaps: Snapshots, val_snaps: Snapshots, *, iters=1500, batch=16384, lr=2e-3, w_pos=4.0,
          miss=1e-3, seed=0, net: E.Network | None = None) -> tuple[E.Network, TrainResult]:
    net = net or E.Network(batch)
    net.set_weights(initial_params(seed))
    gen = torch.Generator().manual_seed(seed + 1)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        smp = random_samples(train_snaps, batch, gen)
        X = train_snaps.features(smp)
        y = train_snaps.labels[smp[:, 0].long(), smp[:, 1].long()].to(torch.float32).contiguous()
        step_lr = lr * (0.5 * (1 + math.cos(math.pi * it / iters)))  # cosine decay
        loss = net.train_step(X, y, w_pos, max(step_lr, 1e-5))
        if it % 100 == 0 or it == iters - 1:
            losses.append((it, float(loss.item())))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    # threshold: at most `miss` of the validation positives fall at or below it
    z = logits_of(net, val_snaps)
    pos = z[val_snaps.labels.bool()]
    thr = float(torch.quantile(pos.float().cpu(), miss).item()) if pos.numel() else 0.0
    pred = z > thr
    lab = val_snaps.labels.bool()
    res = TrainResult(net.get_weights().cpu(), thr, losses, secs,
                      val_recall=float((pred & lab).sum() / max(int(lab.sum()), 1)),
                      val_positive_rate=float(lab.float().mean()),
                      val_predicted_rate=float((pred | lab).float().mean()))
    return net, res


def dilation_radius(K, cfl=0.5):
    """Cells a disturbance can cross in K steps along a diagonal: ceil(K cfl sqrt 2)."""
    return int(math.ceil(K * cfl * math.sqrt(2.0)))


def run(mode, d, *, nx, nv, vmax, steps, K=10, precision=E.FP32, net=None, threshold=0.0, dilation=0,
        timed=False):
    """One run; mode 'plain', 'learned', 'dilated' or 'kinetic' (every cell
    kinetic throughout, the reference of the hybrid).  Returns a dict of
    results (primitives at the end, kinetic cell-steps, judge counters, time)."""
    ind = {"plain": E.IND_PLAIN, "kinetic": E.IND_FROZEN}.get(mode, E.IND_LEARNED)
    cfg = E.make_config(nx, nx, nv, vmax, precision=precision, indicator=ind, scheme=E.ARS233, recon=E.MINMOD2,
                        eta=1e-2, delta=1e-3, learned_k=K)
    eng = E.Engine(cfg)
    if mode == "learned":
        eng.set_learned(net, threshold)
    elif mode == "dilated":
        eng.set_learned(None, 0.0, dilation)
    eng.set_state(d["rho"], d["ux"], d["uy"], d["T"], d["eps"])
    if mode == "kinetic":
        eng.set_mask(np.ones(nx * nx, np.uint8))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eng.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = eng.stats()
    out = dict(prim=np.stack([t.cpu().numpy() for t in eng.moments()]), kinetic_cell_steps=int(st.kinetic_cell_steps),
               seconds=el, mask=eng.mask().cpu().numpy())
    if mode in ("learned", "dilated"):
        out["judge"] = eng.learned_stats()
    return out
