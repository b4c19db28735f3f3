"""Graph-based compression in the library (vbarms_compress_graph, Sec. 2.2, Alg. 1): the
same partition as the oracle, bit for bit, and a working preconditioner on top of it."""
import sys

import numpy as np
import pytest

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


def _no_diagonal(seed):
    # a permutation-like pattern: rows whose blocks hold no diagonal entry
    s = synth.random_pattern_matrix(50, 0.06, twins=10, seed=700 + seed)
    n = s.n
    rows = np.repeat(np.arange(n), np.diff(s.rowptr))
    keep = rows != s.col
    rp, ci, va = synth._csr_from_coo(n, rows[keep], s.col[keep], s.val[keep])
    return synth.System(n, rp, ci, va, np.zeros(n), np.ones(n, np.int32), name=f"nodiag-{seed}")


INPUTS = {
    "grid14": lambda seed: synth.grid_system(7, 6, 5, ell=4, stencil="14rand", perturb=0.15, seed=710 + seed),
    "upwind": lambda seed: synth.upwind_system(8, 7, 6, perturb=0.1, seed=720 + seed),
    "random": lambda seed: synth.random_pattern_matrix(600, 0.01, twins=200, seed=730 + seed),
    "varblock": lambda seed: synth.grid_system(9, 8, 7, ell=6, stencil="7pt", perturb=0.2, seed=740 + seed),
}


@pytest.mark.parametrize("mu", [1.0, 0.9, 0.7, 0.5, 0.3])
@pytest.mark.parametrize("kind", sorted(INPUTS))
def test_graph_compression_matches_oracle(vb, orc, kind, mu):
    for seed in range(2):
        s = INPUTS[kind](seed)
        _say(f"[case] graph compress {kind} seed={seed} n={s.n} nnz={len(s.col)} mu={mu}")
        perm_o, bptr_o = orc.graph_compress(s.n, s.rowptr, s.col, mu)
        sv = vb.Solver()
        rp, ci, va = vb.csr_to_device(s)
        perm, bptr, st = sv.compress_graph(rp, ci, va, mu)
        np.testing.assert_array_equal(perm.cpu().numpy(), perm_o)
        np.testing.assert_array_equal(bptr.cpu().numpy(), bptr_o)
        assert st.nblocks == len(bptr_o) - 1
        assert st.max_block == int(np.diff(bptr_o).max())
        sv.close()


def test_graph_compression_without_diagonal_entries(vb, orc):
    for seed in range(3):
        s = _no_diagonal(seed)
        _say(f"[case] graph compress no-diagonal seed={seed}")
        perm_o, bptr_o = orc.graph_compress(s.n, s.rowptr, s.col, 0.6)
        sv = vb.Solver()
        perm, bptr, _ = sv.compress_graph(*vb.csr_to_device(s), 0.6)
        np.testing.assert_array_equal(perm.cpu().numpy(), perm_o)
        np.testing.assert_array_equal(bptr.cpu().numpy(), bptr_o)
        sv.close()


@pytest.mark.parametrize("levels", [0, 2])
def test_graph_partition_factors_match_oracle_and_solve(vb, orc, levels):
    """The factorization on the graph partition equals the oracle's on the same partition."""
    import torch
    s = synth.grid_system(6, 5, 5, ell=4, stencil="14rand", perturb=0.15, seed=750)
    perm_o, bptr_o = orc.graph_compress(s.n, s.rowptr, s.col, 0.7)
    sv = vb.Solver()
    sv.compress_graph(*vb.csr_to_device(s), 0.7)
    sv.factor(levels, 1e-3)
    o = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm_o, bptr_o, levels, 1e-3)
    assert o.status == 0
    x = np.random.default_rng(3).standard_normal(s.n)
    y = sv.apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    yo = o.apply(x)
    err = np.abs(y - yo).max() / np.abs(yo).max()
    _say(f"[case] graph partition levels={levels}: apply vs oracle {err:.1e}")
    assert err <= 1e-10
    _, info = sv.solve(torch.as_tensor(s.b, device="cuda"), tol=1e-8, restart=30)
    assert info.status == 0 and info.true_relres <= 1e-8
    sv.close()


def test_graph_compression_argument_errors(vb):
    s = synth.grid_system(3, 3, 2, ell=3, stencil="7pt", seed=760)
    sv = vb.Solver()
    dev = vb.csr_to_device(s)
    for mu in (0.0, -0.5, 1.5, float("nan")):
        with pytest.raises(vb.VbarmsError) as e:
            sv.compress_graph(*dev, mu)
        assert e.value.code == vb.ERR_ARG
    sv.close()
