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


def _factor_exports(vb, sv, nlev):
    out = []
    for lvl in range(nlev):
        for w in (vb.M_A, vb.M_AS, vb.M_D, vb.M_G, vb.M_W):
            m = sv.matrix(w, lvl)
            out.append((m.rowptr.copy(), m.colidx.copy(), m.vals.copy()))
    for w in (vb.M_LAST, vb.M_L, vb.M_U, vb.M_DL):
        m = sv.matrix(w)
        out.append((m.rowptr.copy(), m.colidx.copy(), m.vals.copy()))
    return out


@pytest.mark.parametrize("name", ["grid14", "upwind", "random"])
def test_grouped_path_without_merges_equals_one_supernode_per_group(vb, name):
    """group_rows = 1 runs the grouped code path (host greedy, coarse copy, row maps) but no
    neighbour fits, so every group is one supernode: every factor and the application must
    equal, bit for bit, those of the one-supernode path."""
    import torch
    s, tau = SYSTEMS[name]()
    dev = vb.csr_to_device(s)
    res = []
    for g in (0, 1):
        sv = vb.Solver()
        sv.compress(*dev, tau)
        sv.factor(3, 1e-3, group_rows=g)
        x = torch.as_tensor(np.random.default_rng(8).standard_normal(s.n), device="cuda")
        res.append((sv.num_levels(), _factor_exports(vb, sv, sv.num_levels()), sv.apply(x).cpu().numpy(),
                    [sv.level_is(l) for l in range(sv.num_levels())]))
        sv.close()
    assert res[0][0] == res[1][0]
    for a, b in zip(res[0][1], res[1][1]):
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u, v)
    np.testing.assert_array_equal(res[0][2], res[1][2])
    for a, b in zip(res[0][3], res[1][3]):
        np.testing.assert_array_equal(a, b)


def test_groups_on_a_block_diagonal_matrix_empty_the_schur_complement(vb, orc):
    s = synth.random_pattern_matrix(40, 0.0, seed=4)  # diagonal only: every supernode is a group
    perm_o, bptr_o = orc.compress(s.n, s.rowptr, s.col, 1.0)
    o = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm_o, bptr_o, 2, 1e-3, 1, 0, 16)
    sv = vb.Solver()
    sv.compress(*vb.csr_to_device(s), 1.0)
    sv.factor(2, 1e-3, group_rows=16)
    _check_all_factors(vb, orc, o, sv)
    sv.close()


def test_singular_group_reported_like_oracle(vb, orc):
    """A zero pivot row inside a group: the error names the level and the group's smallest
    supernode, as the oracle does."""
    s = synth.grid_system(3, 3, 2, ell=3, stencil="7pt", seed=61)
    val = s.val.copy()
    for r in range(3):
        for k in range(s.rowptr[r], s.rowptr[r + 1]):
            val[k] = 0.0  # node 0's rows vanish
    s.val = val
    perm_o, bptr_o = orc.compress(s.n, s.rowptr, s.col, 1.0)
    o = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm_o, bptr_o, 1, 1e-3, 1, 0, 12)
    assert o.status == orc.ERR_SINGULAR
    sv = vb.Solver()
    sv.compress(*vb.csr_to_device(s), 1.0)
    with pytest.raises(vb.VbarmsError) as e:
        sv.factor(1, 1e-3, group_rows=12)
    assert e.value.code == vb.ERR_SINGULAR
    assert sv.error_location() == (o.err_level, o.err_block)
    sv.close()


def _illconditioned_group(orc, s, gmax, eps=1e-6):
    """The system with the second row of group 0 made equal to its first row on the
    columns of the group, but for eps at the first row's second column, so that the group's
    pivot block is nearly singular (groups follow the pattern, which does not change)."""
    perm, bptr = orc.compress(s.n, s.rowptr, s.col, 1.0)
    o = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm, bptr, 1, 1e-3, 1, 0, gmax)
    members = o.level_is(0)[: o.level_groups(0)[1]]
    cols = set()
    for v in members:
        cols.update(int(perm[k]) for k in range(bptr[v], bptr[v + 1]))
    r0, r1 = int(perm[bptr[members[0]]]), int(perm[bptr[members[0]] + 1])
    val = s.val.copy()
    row0 = {int(s.col[k]): val[k] for k in range(s.rowptr[r0], s.rowptr[r0 + 1])}
    for k in range(s.rowptr[r1], s.rowptr[r1 + 1]):
        c = int(s.col[k])
        if c in cols:
            val[k] = row0.get(c, 0.0)
            if c == r1:
                val[k] += eps * abs(row0[r0])
    from paper_1508_02219_amd.synth import System
    return System(s.n, s.rowptr, s.col, val, s.b, s.node_ell, name=s.name + "-illcond-group")


def test_illconditioned_group_sends_fp32_factorization_to_fp64(vb, orc):
    s = _illconditioned_group(orc, synth.grid_system(5, 4, 4, ell=4, stencil="7pt", seed=93), 16, eps=1e-9)
    perm_o, bptr_o = orc.compress(s.n, s.rowptr, s.col, 1.0)
    o = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm_o, bptr_o, 2, 1e-3, 1, 0, 16)
    assert o.status == 0
    sv = vb.Solver()
    sv.compress(*vb.csr_to_device(s), 1.0)
    sv.factor(2, 1e-3, precision=vb.F32, group_rows=16)
    fs = sv.stats()
    _say(f"[case] ill-conditioned group: {fs.illcond_blocks} blocks below the ratio, fallback {fs.fp64_fallback}")
    assert fs.fp64_fallback == 1 and fs.illcond_blocks >= 1
    _check_all_factors(vb, orc, o, sv)
    sv.close()
