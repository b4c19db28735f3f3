"""GPU checks of the learned parameter selection: MLP kernels and features against the
FP64 references, and what a network trained on the method's own sweeps gains over the
default parameters on held-out matrices."""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as M
from paper_1508_02219_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vb():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_02219_amd import vbarms
    vbarms.lib()
    return vbarms


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dims,batch", [((8, 16, 3, 5), 7), ((3, 4, 2, 2), 5), ((8, 128, 3, 5), 33),
                                        ((6, 5, 0, 3), 4), ((8, 128, 3, 5), 1)])
def test_mlp_kernels_match_fp64_reference(vb, dims, batch):
    _say(f"[case] mlp {dims} batch {batch}")
    rng = np.random.default_rng(sum(dims) + batch)
    net = vb.Mlp(*dims)
    assert net.num_params == M.num_params(*dims)
    p = (rng.standard_normal(net.num_params) * 0.3).astype(np.float32)
    X = rng.standard_normal((batch, dims[0])).astype(np.float32)
    T = rng.standard_normal((batch, dims[3])).astype(np.float32)
    net.set_params(p)
    y = net.forward(X).cpu().numpy()
    yo, _, _ = M.forward(p.astype(float), X.astype(float), *dims)
    assert np.abs(y - yo).max() <= 1e-5 * max(1.0, np.abs(yo).max())
    loss, g = net.loss_grad(X, T)
    lo, go = M.loss_and_grad(p.astype(float), X.astype(float), T.astype(float), *dims)
    assert abs(loss - lo) <= 1e-5 * lo
    assert np.abs(g.cpu().numpy() - go).max() <= 1e-4 * max(1e-3, np.abs(go).max())
    # three Adam steps, each after a fresh gradient
    pp, m1, m2 = p.astype(float), np.zeros(p.size), np.zeros(p.size)
    for k in range(1, 4):
        if k > 1:
            net.loss_grad(X, T, want_grad=False)
        net.adam_step(1e-2)
        _, gk = M.loss_and_grad(pp, X.astype(float), T.astype(float), *dims)
        pp, m1, m2 = M.adam_step(pp, gk, m1, m2, k, 1e-2)
    assert np.abs(net.get_params().cpu().numpy() - pp).max() <= 1e-4


def test_mlp_errors(vb):
    net = vb.Mlp(4, 8, 1, 2)
    with pytest.raises(vb.VbarmsError) as e:
        net.adam_step(1e-3)
    assert e.value.code == vb.ERR_STATE
    net.loss_grad(np.zeros((2, 4)), np.zeros((2, 2)))
    with pytest.raises(vb.VbarmsError) as e:
        net.adam_step(-1.0)
    assert e.value.code == vb.ERR_ARG


@pytest.mark.parametrize("make", [
    lambda: synth.grid_system(6, 5, 4, ell=5, stencil="14rand", perturb=0.1, seed=3),
    lambda: synth.upwind_system(6, 6, 5, pe_range=(0.1, 1000.0), anisotropy=20.0, perturb=0.1, seed=4),
    lambda: synth.random_pattern_matrix(300, 0.02, twins=60, seed=5, diag=6.0),
])
def test_features_match_reference(vb, make):
    s = make()
    _say(f"[case] features {s.name}")
    sv = vb.Solver()
    f = sv.features(*vb.csr_to_device(s))
    fo = M.matrix_features(s.n, s.rowptr, s.col, s.val)
    assert np.allclose(f, fo, rtol=1e-5, atol=1e-6), (f, fo)


def test_learned_parameters_gain_over_defaults(vb):
    """Trains on sweeps the method runs and compares, on held-out matrices, the measured
    time-to-solve at the predicted parameters with the time at the defaults."""
    from paper_1508_02219_amd import learned as Lr
    levels = 3
    taus, tols = (0.7, 0.8, 0.9, 1.0), (1e-4, 1e-3, 1e-2)
    train, test = [], []
    for k in range(14):
        s = Lr.training_system(k, side_range=(5, 8))
        f, res = Lr.sweep(s, levels=levels, taus=taus, tols=tols)
        (test if k >= 10 else train).append((s, f, res))
        _say(f"[case] sweep {k} {s.name} n={s.n}: best "
             f"{min((r for r in res if r.ok), key=lambda r: r.ms).__dict__ if any(r.ok for r in res) else None}")
    X = np.array([f for _, f, _ in train])
    Y = np.array([Lr.label(res, levels) for _, _, res in train])
    pred = Lr.Predictor(levels=levels, seed=0)
    losses = pred.fit(X, Y, epochs=300, lr=3e-3, batch=16)
    assert losses[-1] < losses[0]
    ratios = []
    for s, f, res in test:
        (tau, tl), = pred.predict(f)
        # snap the prediction to the sweep grid and read the measured time there
        tau_g = min(taus, key=lambda v: abs(v - tau))
        t_g = min(tols, key=lambda v: abs(np.log10(v) - np.log10(tl[-1])))
        at = {(r.tau, r.tol): r for r in res}
        got, dflt = at[(tau_g, t_g)], at[(Lr.DEFAULT_TAU, Lr.DEFAULT_TOL)]
        assert got.ok, f"predicted ({tau_g}, {t_g}) did not converge on {s.name}"
        ratios.append(got.ms / dflt.ms if dflt.ok else 0.0)
        _say(f"[case] held-out {s.name}: predicted ({tau_g}, {t_g}) {got.ms:.2f} ms, "
             f"default {dflt.ms if dflt.ok else float('inf'):.2f} ms")
    gain = 1.0 / np.exp(np.mean(np.log(np.maximum(ratios, 1e-3))))
    _say(f"[case] learned parameters: geometric-mean speedup over the defaults {gain:.2f}x")
    assert gain >= 0.95
