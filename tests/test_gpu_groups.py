"""Groups of supernodes in the block independent set (Sec. 2; Sec. 3 Step 3 with block
sparse D_i): the library's groups, pivot blocks, G, W, Schur complements and last-level
factors against the oracle, element by element, and solves through them."""
import sys

import numpy as np
import pytest

from paper_1508_02219_amd import synth
from tests import oracle_helpers as H
from tests.test_gpu_parity import _check_all_factors

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


SYSTEMS = {
    "grid14": lambda: (synth.grid_system(6, 5, 4, ell=4, stencil="14rand", perturb=0.10, seed=801), 0.8),
    "upwind": lambda: (synth.upwind_system(7, 6, 5, seed=802), 1.0),
    "pivoting": lambda: (H.node_rows_reversed(synth.grid_system(5, 4, 4, ell=3, stencil="14rand", seed=803),
                                              "shift"), 1.0),
    "random": lambda: (synth.random_pattern_matrix(300, 0.02, twins=80, seed=804, diag=10.0), 1.0),
}


def _both(vb, orc, name, levels, t, gmax, is_order=0, precision=0):
    s, tau = SYSTEMS[name]()
    _say(f"[case] groups {name} n={s.n} levels={levels} t={t} group_rows={gmax} is_order={is_order} "
         f"precision={precision}")
    perm_o, bptr_o = orc.compress(s.n, s.rowptr, s.col, tau)
    o = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm_o, bptr_o, levels, t, 1, is_order, gmax)
    sv = vb.Solver()
    dev = vb.csr_to_device(s)
    sv.compress(*dev, tau)
    sv.factor(levels, t, 1, precision, is_order, gmax)
    return s, o, sv


@pytest.mark.parametrize("name", sorted(SYSTEMS))
@pytest.mark.parametrize("levels,t,gmax", [(1, 1e-3, 16), (3, 1e-4, 24), (2, 0.0, 32), (3, 1e-3, 12)])
def test_group_factors_match_oracle(vb, orc, name, levels, t, gmax):
    s, o, sv = _both(vb, orc, name, levels, t, gmax)
    assert o.status == 0
    for lvl in range(o.nlevels):
        np.testing.assert_array_equal(sv.level_groups(lvl), o.level_groups(lvl))
    assert any(np.diff(o.level_groups(l)).max() > 1 for l in range(o.nlevels))
    _check_all_factors(vb, orc, o, sv)
    sv.close()


@pytest.mark.parametrize("name", ["grid14", "upwind"])
def test_weighted_groups_match_oracle(vb, orc, name):
    s, o, sv = _both(vb, orc, name, 3, 1e-3, 20, is_order=1)
    assert o.status == 0
    for lvl in range(o.nlevels):
        np.testing.assert_array_equal(sv.level_groups(lvl), o.level_groups(lvl))
    _check_all_factors(vb, orc, o, sv)
    sv.close()


@pytest.mark.parametrize("gmax", [16, 32])
def test_group_apply_and_solve(vb, orc, gmax):
    import torch
    s, o, sv = _both(vb, orc, "upwind", 3, 1e-3, gmax)
    x = np.random.default_rng(5).standard_normal(s.n)
    y = sv.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    yo = o.apply(x)
    bad = np.abs(y - yo) > 1e-10 * np.abs(yo) + 1e-14 * np.abs(yo).max()
    assert not bad.any(), np.abs(y - yo).max()
    _, info = sv.solve(torch.as_tensor(s.b, device="cuda"), tol=1e-8, restart=30)
    _say(f"[case] group_rows={gmax}: {info.iters} iterations, true relres {info.true_relres:.2e}")
    assert info.status == 0 and info.true_relres <= 1e-8
    sv.close()


def test_group_factors_in_float32(vb, orc):
    """FP32 factors with groups: the application stays close to the FP64 oracle's and the
    FP64 FGMRES still reaches 1e-8."""
    import torch
    s, o, sv = _both(vb, orc, "grid14", 2, 1e-4, 24, precision=1)
    x = np.random.default_rng(6).standard_normal(s.n)
    y = sv.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    yo = o.apply(x)
    e = np.abs(y - yo).max() / np.abs(yo).max()
    _say(f"[case] fp32 groups apply error vs fp64 oracle {e:.1e}")
    assert e <= 1e-4
    _, info = sv.solve(torch.as_tensor(s.b, device="cuda"), tol=1e-8, restart=30)
    assert info.status == 0 and info.true_relres <= 1e-8
    sv.close()


def test_group_rows_argument_errors(vb):
    s = synth.grid_system(3, 3, 2, ell=3, stencil="7pt", seed=805)
    sv = vb.Solver()
    sv.compress(*vb.csr_to_device(s), 1.0)
    for g in (-1, 33):
        with pytest.raises(vb.VbarmsError) as e:
            sv.factor(1, 1e-3, group_rows=g)
        assert e.value.code == vb.ERR_ARG
    sv.close()
