"""Batches of independent systems (vbarms_batch_*): the combined factorization gives every
system exactly its own factors, and the lockstep FGMRES reaches the tolerance per system
and right-hand side."""
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


def _systems():
    # uneven sizes, block sizes 3, 5, 6 and 1..7, different stencils and perturbations
    return [synth.grid_system(6, 5, 4, ell=3, stencil="14rand", perturb=0.1, seed=501),
            synth.grid_system(8, 7, 6, ell=5, stencil="14rand", perturb=0.1, seed=502),
            synth.upwind_system(5, 5, 4, seed=503),
            synth.grid_system(3, 3, 2, ell=6, stencil="7pt", seed=504),
            synth.upwind_system(7, 6, 6, ell_choices=(5,), pe_range=(1.0, 50.0), perturb=0.05, seed=505)]


def _residual(s, x):
    import scipy.sparse as sp
    a = sp.csr_matrix((s.val, s.col, s.rowptr), shape=(s.n, s.n))
    return np.linalg.norm(s.b - a @ x) / np.linalg.norm(s.b)


@pytest.mark.parametrize("tau,levels,t,groups", [(0.8, 2, 1e-3, 0), (1.0, 0, 1e-3, 0), (0.8, 3, 1e-4, 0),
                                                 (0.8, 2, 1e-3, 16), (1.0, 3, 1e-4, 32)])
def test_batch_factors_are_the_individual_factors(vb, tau, levels, t, groups):
    """M^{-1} of the combined system applied to a concatenated vector equals, bit for bit,
    every system's own M^{-1} applied to its part (groups never span two systems)."""
    import torch
    systems = _systems()
    _say(f"[case] batch of {len(systems)} systems tau={tau} levels={levels} t={t} group_rows={groups}")
    bs = vb.BatchSolver()
    off = bs.factor([vb.csr_to_device(s) for s in systems], tau, levels, t, group_rows=groups)
    assert list(np.diff(off)) == [s.n for s in systems]
    x = np.random.default_rng(1).standard_normal(int(off[-1]))
    y = bs.handle().apply(torch.as_tensor(x, device="cuda")).cpu().numpy()
    for q, s in enumerate(systems):
        sv = vb.Solver()
        sv.compress(*vb.csr_to_device(s), tau)
        sv.factor(levels, t, group_rows=groups)
        yq = sv.apply(torch.as_tensor(x[off[q]:off[q + 1]].copy(), device="cuda")).cpu().numpy()
        assert np.array_equal(y[off[q]:off[q + 1]], yq), f"system {q}"
        sv.close()
    bs.close()


def test_batch_solve_reaches_tolerance_per_system_and_rhs(vb):
    import torch
    systems = _systems()
    bs = vb.BatchSolver()
    off = bs.factor([vb.csr_to_device(s) for s in systems], 0.8, 2, 1e-3)
    N = int(off[-1])
    rng = np.random.default_rng(7)
    # column 0: every system's own b = A 1; columns 1-2: N(0,1); system 3 of column 2 is zero
    B = np.concatenate([s.b for s in systems])[None, :].repeat(3, axis=0)
    B[1:] = rng.standard_normal((2, N))
    B[2, off[3]:off[4]] = 0.0
    X, info = bs.solve(torch.as_tensor(B, device="cuda"), tol=1e-8, restart=20)
    X = X.cpu().numpy()
    for r in range(3):
        for q, s in enumerate(systems):
            inf = info[r][q]
            if r == 2 and q == 3:
                assert inf.status == 0 and np.all(X[r, off[q]:off[q + 1]] == 0.0)
                continue
            s_r = synth.System(s.n, s.rowptr, s.col, s.val, B[r, off[q]:off[q + 1]], s.node_ell)
            rel = _residual(s_r, X[r, off[q]:off[q + 1]])
            assert inf.status == 0 and rel <= 1e-8 and abs(rel - inf.true_relres) <= 1e-10 * max(1.0, rel) + 1e-15
    # iteration counts agree with single-system solves (same factors; only the summation
    # order of the inner products differs)
    for q, s in enumerate(systems):
        sv = vb.Solver()
        sv.compress(*vb.csr_to_device(s), 0.8)
        sv.factor(2, 1e-3)
        _, i1 = sv.solve(torch.as_tensor(s.b, device="cuda"), tol=1e-8, restart=20)
        _say(f"[case] system {q}: batch its {info[0][q].iters}, alone {i1.iters}")
        assert abs(info[0][q].iters - i1.iters) <= 1
        sv.close()
    bs.close()


def test_batch_iteration_limit_reports_not_converged(vb):
    import torch
    systems = _systems()[:3]
    bs = vb.BatchSolver()
    off = bs.factor([vb.csr_to_device(s) for s in systems], 0.8, 1, 5e-2)
    B = torch.as_tensor(np.concatenate([s.b for s in systems])[None, :], device="cuda")
    X, info = bs.solve(B, tol=1e-12, restart=3, maxit=2)
    assert all(i.status == vb.NOT_CONVERGED and i.iters <= 2 for i in info[0])
    bs.close()


def test_batch_argument_errors(vb):
    import torch
    bs = vb.BatchSolver()
    with pytest.raises(vb.VbarmsError) as e:
        bs.solve(torch.zeros((1, 4), dtype=torch.float64, device="cuda"))
    assert e.value.code in (vb.ERR_STATE, vb.ERR_ARG)
    with pytest.raises(vb.VbarmsError) as e:
        bs.factor([], 0.8, 1, 1e-3)
    assert e.value.code == vb.ERR_ARG
    bs.close()


def test_batch_right_hand_sides_in_lockstep_equal_one_at_a_time(vb):
    """Several right-hand sides go through one lockstep FGMRES (multi-vector SpMV and
    preconditioner); every solution equals, bit for bit, the solve of its right-hand side
    alone, and so do the iteration counts."""
    import torch
    systems = _systems()[:4]
    bs = vb.BatchSolver()
    off = bs.factor([vb.csr_to_device(s) for s in systems], 0.8, 2, 1e-3, group_rows=16)
    N = int(off[-1])
    B = np.random.default_rng(21).standard_normal((5, N))
    B[3, off[1]:off[2]] = 0.0
    X, info = bs.solve(torch.as_tensor(B, device="cuda"), tol=1e-8, restart=15)
    X = X.cpu().numpy()
    for r in range(5):
        Xr, ir = bs.solve(torch.as_tensor(B[r:r + 1].copy(), device="cuda"), tol=1e-8, restart=15)
        assert np.array_equal(X[r], Xr.cpu().numpy()[0]), f"right-hand side {r}"
        for q in range(len(systems)):
            assert info[r][q].iters == ir[0][q].iters and info[r][q].status == ir[0][q].status
            assert info[r][q].true_relres == ir[0][q].true_relres
    bs.close()
