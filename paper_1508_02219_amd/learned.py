"""Learned selection of tau and the per-level drop tolerances (a project extension).

The paper tunes the compression threshold tau by hand per matrix (Table 3) and prints no
drop tolerance; this module predicts both from features of the matrix.  Everything
numeric runs in the library: features (``vbarms_features``), the sweeps that label the
training matrices (compress + factor + FGMRES on the GPU), and the network's forward pass,
backpropagation and Adam update (``vbarms_mlp_*``).  This file only orchestrates.

Label of a matrix: the (tau, t) of the sweep grid with the smallest measured
time-to-solve among the settings that reach the tolerance.  Target vector:
[tau, log10 t_0, ..., log10 t_L] (the sweep uses one t for every level).  Without a
trained network the defaults tau = 0.7 and t = 1e-4 apply.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import synth
from . import vbarms as V

TAUS = (0.6, 0.7, 0.8, 0.9, 1.0)
TOLS = (1e-5, 1e-4, 1e-3, 1e-2)
DEFAULT_TAU, DEFAULT_TOL = 0.7, 1e-4
HIDDEN, DEPTH = 128, 3


@dataclass
class RunResult:
    tau: float
    tol: float
    ok: bool
    iters: int
    ms: float          # compress + factor + solve, device time
    relres: float


def training_system(seed: int, side_range=(6, 10)):
    """A matrix of the training distribution: upwind grid, fixed block size per matrix,
    Peclet LogUniform(0.1, 1000), anisotropy 1..100 on z-links, 0-20% block perturbation."""
    rng = np.random.default_rng(10_000 + seed)
    side = int(rng.integers(side_range[0], side_range[1] + 1))
    ell = int(rng.choice([4, 5, 6]))
    aniso = float(np.exp(rng.uniform(0.0, np.log(100.0))))
    pert = float(rng.uniform(0.0, 0.2))
    return synth.upwind_system(side, side, side, ell_choices=(ell,), pe_range=(0.1, 1000.0), anisotropy=aniso,
                               perturb=pert, seed=seed)


def run_once(sv: V.Solver, dev, b, tau, tol, levels, restart, rtol, maxit) -> RunResult:
    try:
        sv.compress(*dev, tau)
        sv.factor(levels, tol)
        _, info = sv.solve(b, tol=rtol, restart=restart, maxit=maxit)
    except V.VbarmsError:
        return RunResult(tau, tol, False, 0, math.inf, math.inf)
    st = sv.stats()
    ok = info.status == 0 and info.true_relres <= rtol
    return RunResult(tau, tol, ok, info.iters, st.compress_ms + st.factor_ms + st.solve_ms, info.true_relres)


def sweep(system, levels=3, restart=50, rtol=1e-8, maxit=400, taus=TAUS, tols=TOLS, repeats=1):
    """Runs every (tau, t) of the grid on one system; returns (features, [RunResult])."""
    import torch
    sv = V.Solver()
    dev = V.csr_to_device(system)
    b = torch.as_tensor(system.b, device="cuda")
    feats = sv.features(*dev)
    res = []
    for tau in taus:
        for tol in tols:
            best = None
            for _ in range(repeats):
                r = run_once(sv, dev, b, tau, tol, levels, restart, rtol, maxit)
                best = r if best is None or r.ms < best.ms else best
            res.append(best)
    sv.close()
    return feats, res


def label(results, levels):
    ok = [r for r in results if r.ok]
    if not ok:
        tau, tol = DEFAULT_TAU, DEFAULT_TOL
    else:
        r = min(ok, key=lambda r: r.ms)
        tau, tol = r.tau, r.tol
    return np.array([tau] + [math.log10(tol)] * (levels + 1), dtype=np.float32)


class Predictor:
    """Feature normalization + the MLP; predicts (tau, [t_0..t_L])."""

    def __init__(self, levels=3, seed=0):
        self.levels = levels
        self.net = V.Mlp(V.NFEAT, HIDDEN, DEPTH, levels + 2)
        rng = np.random.default_rng(seed)
        # He initialization of every weight matrix, zero biases (drawn here, passed in)
        p = np.zeros(self.net.num_params, np.float32)
        off = 0
        dims = [V.NFEAT] + [HIDDEN] * DEPTH + [levels + 2]
        for i, o in zip(dims[:-1], dims[1:]):
            p[off:off + o * i] = rng.standard_normal(o * i) * math.sqrt(2.0 / i)
            off += o * i + o
        self.net.set_params(p)
        self.mu = np.zeros(V.NFEAT, np.float32)
        self.sd = np.ones(V.NFEAT, np.float32)
        self.ymu = np.zeros(levels + 2, np.float32)
        self.ysd = np.ones(levels + 2, np.float32)

    def fit(self, X, Y, epochs=400, lr=3e-3, batch=64, seed=0):
        X = np.asarray(X, np.float32)
        Y = np.asarray(Y, np.float32)
        self.mu, self.sd = X.mean(0), X.std(0) + 1e-6
        self.ymu, self.ysd = Y.mean(0), Y.std(0) + 1e-3
        Xn, Yn = (X - self.mu) / self.sd, (Y - self.ymu) / self.ysd
        rng = np.random.default_rng(seed)
        losses = []
        for ep in range(epochs):
            order = rng.permutation(len(Xn))
            for s in range(0, len(order), batch):
                idx = order[s:s + batch]
                loss, _ = self.net.loss_grad(Xn[idx], Yn[idx], want_grad=False)
                self.net.adam_step(lr)
                losses.append(loss)
        return losses

    def predict(self, feats):
        x = ((np.atleast_2d(np.asarray(feats, np.float32)) - self.mu) / self.sd).astype(np.float32)
        y = self.net.forward(x).cpu().numpy() * self.ysd + self.ymu
        out = []
        for row in y:
            tau = float(np.clip(row[0], 0.5, 1.0))
            tols = [float(10.0 ** np.clip(v, -8.0, -1.0)) for v in row[1:]]
            out.append((tau, tols))
        return out
