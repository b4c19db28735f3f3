"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: brute force on tiny
inputs, closed forms, exact algebraic identities at zero dropping, or library routines
for the special cases that reduce to them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1508_02219_amd import synth
from tests import oracle_helpers as H


def _oracle(O, s, tau, levels, droptol, drop_schur=1):
    perm, bptr = O.compress(s.n, s.rowptr, s.col, tau)
    return O.Oracle(s.n, s.rowptr, s.col, s.val, perm, bptr, levels, droptol, drop_schur), perm, bptr


def _split(bm, is_list):
    """Scalar index sets of independent-set blocks and of the rest (both ascending)."""
    isb = set(int(i) for i in is_list)
    rows_is = np.concatenate([np.arange(bm.rb[i], bm.rb[i + 1]) for i in sorted(isb)] or [np.zeros(0, int)])
    rest = [i for i in range(bm.p) if i not in isb]
    rows_rest = np.concatenate([np.arange(bm.rb[i], bm.rb[i + 1]) for i in rest] or [np.zeros(0, int)])
    return rows_is.astype(int), rows_rest.astype(int)


def _block_lu_parts(dm):
    """From an exported pivot-block matrix: dense block diagonals P^T L and U."""
    n = dm.rb[-1]
    PtL = np.zeros((n, n))
    Uu = np.zeros((n, n))
    for i in range(dm.p):
        a, b = dm.rb[i], dm.rb[i + 1]
        m = b - a
        lu = dm.block(i)
        Lm = np.tril(lu, -1) + np.eye(m)
        Um = np.triu(lu)
        P = np.eye(m)
        for k in range(m):
            pk = dm.piv[a + k]
            P[[k, pk]] = P[[pk, k]]
        PtL[a:b, a:b] = P.T @ Lm
        Uu[a:b, a:b] = Um
    return PtL, Uu


# --------------------------------------------------------------------------------------
# Compression (Sec. 2.1)
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_tau_one_gives_identical_pattern_classes(orc, seed):
    s = synth.random_pattern_matrix(90, 0.06, twins=30, seed=seed)
    perm, bptr = orc.compress(s.n, s.rowptr, s.col, 1.0)
    p2, b2 = H.identical_pattern_partition(s.n, s.rowptr, s.col)
    np.testing.assert_array_equal(perm, p2)
    np.testing.assert_array_equal(bptr, b2)


def test_empty_rows_stay_singletons(orc):
    n = 6
    rowptr = np.array([0, 0, 2, 2, 4, 4, 4], dtype=np.int64)  # rows 0, 2, 4, 5 empty
    col = np.array([1, 3, 1, 3], dtype=np.int32)
    perm, bptr = orc.compress(n, rowptr, col, 0.5)
    np.testing.assert_array_equal(perm, [0, 1, 3, 2, 4, 5])
    np.testing.assert_array_equal(bptr, [0, 1, 3, 4, 5, 6])


@pytest.mark.parametrize("tau", [0.3183, 0.5772, 0.7071, 0.9133])
@pytest.mark.parametrize("seed", [5, 6])
def test_angle_compression_matches_bruteforce(orc, tau, seed):
    s = synth.random_pattern_matrix(140, 0.05, twins=25, seed=seed)
    perm, bptr = orc.compress(s.n, s.rowptr, s.col, tau)
    p2, b2, margin = H.angle_partition_bruteforce(s.n, s.rowptr, s.col, tau)
    assert margin > 1e-9
    np.testing.assert_array_equal(perm, p2)
    np.testing.assert_array_equal(bptr, b2)


def test_angle_compression_on_perturbed_stencil_matches_bruteforce(orc):
    s = synth.grid_system(3, 3, 3, ell=5, stencil="14rand", perturb=0.10, seed=7)
    for tau in (0.61, 0.8, 0.93):
        perm, bptr = orc.compress(s.n, s.rowptr, s.col, tau)
        p2, b2, margin = H.angle_partition_bruteforce(s.n, s.rowptr, s.col, tau)
        assert margin > 1e-9
        np.testing.assert_array_equal(perm, p2)
        np.testing.assert_array_equal(bptr, b2)


def test_perfect_blocks_recovered(orc):
    s = synth.grid_system(4, 3, 3, ell=4, stencil="7pt", seed=3)
    perm, bptr = orc.compress(s.n, s.rowptr, s.col, 1.0)
    np.testing.assert_array_equal(perm, np.arange(s.n))
    np.testing.assert_array_equal(bptr, np.arange(0, s.n + 1, 4))
    o = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm, bptr, 0, 0.0)
    a = o.matrix(orc.LAST)
    cells = sum((a.rb[i + 1] - a.rb[i]) * (a.cb[a.colidx[k] + 1] - a.cb[a.colidx[k]])
                for i in range(a.p) for k in range(a.rowptr[i], a.rowptr[i + 1]))
    assert cells == s.nnz  # average block density 1


def test_twin_nodes_merge(orc):
    # two mutually coupled nodes are indistinguishable: one block of 2*ell rows
    s = synth.grid_system(1, 1, 2, ell=3, stencil="7pt", seed=1)
    perm, bptr = orc.compress(s.n, s.rowptr, s.col, 1.0)
    np.testing.assert_array_equal(bptr, [0, 6])


def test_tau_one_relabel_invariant(orc):
    s = synth.random_pattern_matrix(80, 0.07, twins=20, seed=11)
    rng = np.random.default_rng(0)
    q = rng.permutation(s.n)  # new index k holds old row q[k]
    a = s.dense()
    pat = a != 0
    ap = a[np.ix_(q, q)]
    pp = pat[np.ix_(q, q)]
    rows, cols = np.nonzero(pp)
    rowptr = np.zeros(s.n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    perm1, bptr1 = orc.compress(s.n, s.rowptr, s.col, 1.0)
    perm2, bptr2 = orc.compress(s.n, rowptr, cols.astype(np.int32), 1.0)
    g1 = {frozenset(perm1[bptr1[i]:bptr1[i + 1]].tolist()) for i in range(len(bptr1) - 1)}
    g2 = {frozenset(q[perm2[bptr2[i]:bptr2[i + 1]]].tolist()) for i in range(len(bptr2) - 1)}
    assert g1 == g2
    del ap


def test_compress_rejects_bad_tau(orc):
    s = synth.random_pattern_matrix(10, 0.2, seed=1)
    for tau in (0.0, -0.5, 1.5, float("nan")):
        with pytest.raises(ValueError):
            orc.compress(s.n, s.rowptr, s.col, tau)


# --------------------------------------------------------------------------------------
# Independent set (Sec. 2, Sec. 3 Step 3)
# --------------------------------------------------------------------------------------
def test_independent_set_checkerboard_closed_form(orc):
    s = synth.config_system(1)
    o, perm, bptr = _oracle(orc, s, 1.0, 1, 1e-3)
    nodes = np.arange(1000)
    x, y, z = nodes % 10, (nodes // 10) % 10, nodes // 100
    expect = nodes[(x + y + z) % 2 == 0]
    np.testing.assert_array_equal(o.level_is(0), expect)
    assert len(expect) == 500


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_independent_set_matches_bruteforce_all_levels(orc, seed):
    s = synth.random_pattern_matrix(150, 0.03, twins=20, seed=seed + 20, diag=6.0)
    o, perm, bptr = _oracle(orc, s, 0.6, 3, 1e-3)
    assert o.status == 0
    for lvl in range(o.nlevels):
        a = o.matrix(orc.AS, lvl)
        adj = H.quotient_adjacency(a)
        is_list = o.level_is(lvl)
        np.testing.assert_array_equal(is_list, H.greedy_is_bruteforce(adj))
        iset = set(is_list.tolist())
        for v in iset:  # independent
            assert not (adj[v] & iset)
        for v in range(a.p):  # maximal
            assert v in iset or (adj[v] & iset)


# --------------------------------------------------------------------------------------
# Scaling (Sec. 3 Step 2)
# --------------------------------------------------------------------------------------
def test_scaling_unit_maxima(orc):
    s = synth.grid_system(3, 3, 4, ell=3, stencil="14rand", perturb=0.1, seed=4)
    o, perm, bptr = _oracle(orc, s, 0.8, 2, 1e-3)
    for lvl in range(o.nlevels):
        a = o.matrix(orc.A, lvl).dense()
        asd = o.matrix(orc.AS, lvl).dense()
        s1, s2 = o.level_scaling(lvl)
        np.testing.assert_array_equal(s1, 1.0 / np.abs(a).max(axis=1))
        cmax = np.abs(asd).max(axis=0)
        rmax = np.abs(asd).max(axis=1)
        assert np.all(np.abs(cmax - 1.0) <= 4e-16)
        assert np.all(rmax <= 1.0 + 4e-16)
        np.testing.assert_allclose(asd, (s1[:, None] * a) * s2[None, :], rtol=0, atol=0)


# --------------------------------------------------------------------------------------
# Partial block factorization (Sec. 3 Step 4, Eq. vbarms, Eq. schurcomp)
# --------------------------------------------------------------------------------------
def test_pivot_blocks_match_lapack_getrf(orc):
    s = synth.grid_system(4, 4, 3, ell=5, stencil="14rand", seed=9)
    o, perm, bptr = _oracle(orc, s, 1.0, 1, 1e-3)
    asd = o.matrix(orc.AS, 0)
    dm = o.matrix(orc.D, 0)
    for t, i in enumerate(o.level_is(0)):
        k = [kk for kk in range(asd.rowptr[i], asd.rowptr[i + 1]) if asd.colidx[kk] == i][0]
        lu, piv = sla.lu_factor(asd.block(k))
        np.testing.assert_array_equal(dm.piv[dm.rb[t]:dm.rb[t + 1]], piv)
        np.testing.assert_allclose(dm.block(t), lu, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("system", ["grid", "rand"])
def test_zero_drop_schur_and_factorization_identity(orc, system):
    if system == "grid":
        s = synth.grid_system(4, 3, 3, ell=4, stencil="14rand", perturb=0.1, seed=12)
        tau = 0.8
    else:
        s = synth.random_pattern_matrix(120, 0.04, twins=30, seed=13, diag=8.0)
        tau = 0.55
    o, perm, bptr = _oracle(orc, s, tau, 1, 0.0)
    assert o.status == 0
    As = o.matrix(orc.AS, 0)
    a = As.dense()
    ri, rr = _split(As, o.level_is(0))
    D, F, E, Cm = a[np.ix_(ri, ri)], a[np.ix_(ri, rr)], a[np.ix_(rr, ri)], a[np.ix_(rr, rr)]
    S_exact = Cm - E @ np.linalg.solve(D, F)
    S = o.matrix(orc.LAST).dense()
    scale = np.abs(S_exact).max()
    assert np.abs(S - S_exact).max() <= 1e-12 * scale
    # Eq. vbarms: [D F; E C] = [P^T L 0; W I] [U G; 0 S]
    PtL, Uu = _block_lu_parts(o.matrix(orc.D, 0))
    G = o.matrix(orc.G, 0).dense()
    Wm = o.matrix(orc.W, 0).dense()
    ni, nr = len(ri), len(rr)
    left = np.block([[PtL, np.zeros((ni, nr))], [Wm, np.eye(nr)]])
    right = np.block([[Uu, G], [np.zeros((nr, ni)), S]])
    full = np.block([[D, F], [E, Cm]])
    assert np.abs(left @ right - full).max() <= 1e-12 * np.abs(full).max()


def test_dropping_matches_dense_bruteforce(orc):
    s = synth.grid_system(4, 4, 4, ell=3, stencil="14rand", perturb=0.1, seed=21)
    t = 0.012
    o, perm, bptr = _oracle(orc, s, 0.8, 1, [t, 0.0])
    assert o.status == 0
    As = o.matrix(orc.AS, 0)
    is_list = o.level_is(0)
    isset = set(is_list.tolist())
    rest = [i for i in range(As.p) if i not in isset]
    num = {int(b): k for k, b in enumerate(is_list)}
    num.update({b: k for k, b in enumerate(rest)})
    dm = o.matrix(orc.D, 0)
    PtL, Uu = _block_lu_parts(dm)
    margins = []
    # expected G, W blocks (dense per block), applying the drop rule
    Gx, Wx = {}, {}
    nF = nE = 0
    for i in range(As.p):
        for k in range(As.rowptr[i], As.rowptr[i + 1]):
            j = int(As.colidx[k])
            blk = As.block(k)
            if i in isset and j not in isset:
                nF += 1
                a, b = dm.rb[num[i]], dm.rb[num[i] + 1]
                val = np.linalg.solve(PtL[a:b, a:b], blk)
                r = H.block_sumsq_ratio(val, t)
                margins.append(abs(r - 1))
                if r >= 1:
                    Gx[(num[i], num[j])] = val
            if i not in isset and j in isset:
                nE += 1
                a, b = dm.rb[num[j]], dm.rb[num[j] + 1]
                val = np.linalg.solve(Uu[a:b, a:b].T, blk.T).T
                r = H.block_sumsq_ratio(val, t)
                margins.append(abs(r - 1))
                if r >= 1:
                    Wx[(num[i], num[j])] = val
    assert min(margins) > 1e-9
    G, Wm = o.matrix(orc.G, 0), o.matrix(orc.W, 0)

    def blocks(bm):
        return {(i, int(bm.colidx[k])): bm.block(k) for i in range(bm.p)
                for k in range(bm.rowptr[i], bm.rowptr[i + 1])}

    gb, wb = blocks(G), blocks(Wm)
    assert set(gb) == set(Gx) and set(wb) == set(Wx)
    assert 0 < len(gb) < nF and 0 < len(wb) < nE  # the threshold both keeps and drops
    for key in Gx:
        np.testing.assert_allclose(gb[key], Gx[key], rtol=1e-12, atol=1e-14)
    for key in Wx:
        np.testing.assert_allclose(wb[key], Wx[key], rtol=1e-12, atol=1e-14)
    # Schur with dropped W, G blocks, then off-diagonal dropping
    nr = len(rest)
    rsz = [As.rb[b + 1] - As.rb[b] for b in rest]
    Sx = {}
    n_before = 0
    for jn, J in enumerate(rest):
        acc = {}
        for k in range(As.rowptr[J], As.rowptr[J + 1]):
            K = int(As.colidx[k])
            if K not in isset:
                acc[num[K]] = As.block(k).copy()
        for (wj, wi), wv in sorted(Wx.items()):
            if wj != jn:
                continue
            for (gi, gk), gv in sorted(Gx.items()):
                if gi != wi:
                    continue
                acc.setdefault(gk, np.zeros((rsz[jn], rsz[gk])))
                acc[gk] = acc[gk] - wv @ gv
        n_before += len(acc)
        for K, v in acc.items():
            r = H.block_sumsq_ratio(v, t)
            if K == jn or r >= 1:
                Sx[(jn, K)] = v
            if K != jn:
                margins.append(abs(r - 1))
    assert min(margins) > 1e-9
    sb = blocks(o.matrix(orc.LAST))
    assert set(sb) == set(Sx)
    assert nr < len(sb) < n_before
    for key in Sx:
        np.testing.assert_allclose(sb[key], Sx[key], rtol=1e-11, atol=1e-13)


def test_no_schur_drop_mode_keeps_all_blocks(orc):
    s = synth.grid_system(4, 4, 3, ell=3, stencil="14rand", perturb=0.1, seed=22)
    o1, _, _ = _oracle(orc, s, 0.8, 1, [0.05, 0.0], drop_schur=1)
    o0, _, _ = _oracle(orc, s, 0.8, 1, [0.05, 0.0], drop_schur=0)
    a1, a0 = o1.matrix(orc.LAST), o0.matrix(orc.LAST)
    assert a0.nb > a1.nb
    d0 = a0.dense()
    d1 = a1.dense()
    kept = d1 != 0
    np.testing.assert_array_equal(d0[kept], d1[kept])


def _weighted_greedy_bruteforce(bm):
    """Greedy independent set on the quotient graph of A + A^T visiting block rows by
    descending ||A_II||_F / sum_J ||A_IJ||_F (ties ascending), from the dense blocks; also
    returns the smallest relative gap between distinct weights (to rule out near ties)."""
    w = np.zeros(bm.p)
    for i in range(bm.p):
        norms = {int(bm.colidx[k]): np.linalg.norm(bm.block(k)) for k in range(bm.rowptr[i], bm.rowptr[i + 1])}
        tot = sum(norms.values())
        w[i] = norms.get(i, 0.0) / tot if tot > 0 else 0.0
    order = sorted(range(bm.p), key=lambda i: (-w[i], i))
    adj = H.quotient_adjacency(bm)
    marked = np.zeros(bm.p, bool)
    out = []
    for v in order:
        if marked[v]:
            continue
        out.append(v)
        marked[v] = True
        for u in adj[v]:
            marked[u] = True
    ws = np.sort(w)
    gaps = np.diff(ws)
    gaps = gaps[gaps > 0]
    return np.array(sorted(out), dtype=np.int32), (gaps.min() / ws.max() if gaps.size else np.inf), adj


@pytest.mark.parametrize("levels", [1, 3])
@pytest.mark.parametrize("maker", ["grid", "upwind"])
def test_weighted_independent_set_matches_bruteforce(orc, maker, levels):
    """Sec. 3 Step 3, weighted greedy: brute force on every level, independence and
    maximality, and a different set from the natural order on the same input."""
    if maker == "grid":
        s = synth.grid_system(5, 4, 4, ell=4, stencil="14rand", perturb=0.1, seed=91)
        tau = 0.8
    else:
        s = synth.upwind_system(5, 4, 4, seed=92)
        tau = 1.0
    perm, bptr = orc.compress(s.n, s.rowptr, s.col, tau)
    o = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm, bptr, levels, 1e-3, 1, 1)
    on = orc.Oracle(s.n, s.rowptr, s.col, s.val, perm, bptr, levels, 1e-3, 1, 0)
    assert o.status == 0 and o.nlevels == levels
    for lvl in range(levels):
        As = o.matrix(orc.AS, lvl)
        want, gap, adj = _weighted_greedy_bruteforce(As)
        assert gap > 1e-9
        got = o.level_is(lvl)
        np.testing.assert_array_equal(got, want)
        isset = set(got.tolist())
        assert all(not (adj[v] & isset) for v in isset)
        assert all(v in isset or (adj[v] & isset) for v in range(As.p))
    assert not np.array_equal(o.level_is(0), on.level_is(0))


# --------------------------------------------------------------------------------------
# Groups of nodes in the block independent set (Sec. 2; Sec. 3 Step 3, D_i block sparse)
# --------------------------------------------------------------------------------------
_GROUP_INPUTS = {
    "grid": (lambda: synth.grid_system(5, 4, 4, ell=4, stencil="14rand", perturb=0.1, seed=93), 0.8),
    "upwind": (lambda: synth.upwind_system(5, 5, 4, seed=94), 1.0),
    "random": (lambda: synth.random_pattern_matrix(160, 0.03, twins=30, seed=95, diag=6.0), 0.6),
}


def _group_oracle(orc, maker, levels, t, gmax, is_order=0):
    mk, tau = _GROUP_INPUTS[maker]
    s = mk()
    perm, bptr = orc.compress(s.n, s.rowptr, s.col, tau)
    return s, orc.Oracle(s.n, s.rowptr, s.col, s.val, perm, bptr, levels, t, 1, is_order, gmax)


def _groups_of(o, lvl):
    is_list, gptr = o.level_is(lvl), o.level_groups(lvl)
    return [is_list[gptr[g]:gptr[g + 1]].tolist() for g in range(len(gptr) - 1)]


def _weights_order(bm):
    w = np.zeros(bm.p)
    for i in range(bm.p):
        norms = {int(bm.colidx[k]): np.linalg.norm(bm.block(k)) for k in range(bm.rowptr[i], bm.rowptr[i + 1])}
        tot = sum(norms.values())
        w[i] = norms.get(i, 0.0) / tot if tot > 0 else 0.0
    return sorted(range(bm.p), key=lambda i: (-w[i], i))


@pytest.mark.parametrize("is_order", [0, 1])
@pytest.mark.parametrize("gmax", [12, 20, 32])
@pytest.mark.parametrize("maker", sorted(_GROUP_INPUTS))
def test_group_independent_sets_match_bruteforce(orc, maker, gmax, is_order):
    """Every level: the groups of a set-based restatement of the greedy; no coupling between
    two groups; every remaining supernode next to a group; members next to the group's
    opener; groups within gmax rows unless the opener alone is larger."""
    s, o = _group_oracle(orc, maker, 3, 1e-3, gmax, is_order)
    assert o.status == 0
    merged = 0
    for lvl in range(o.nlevels):
        a = o.matrix(orc.AS, lvl)
        adj = H.quotient_adjacency(a)
        sizes = np.diff(a.rb)
        order = _weights_order(a) if is_order else None
        got = _groups_of(o, lvl)
        assert got == H.greedy_groups_bruteforce(adj, sizes, gmax, order)
        owner = {v: g for g, mem in enumerate(got) for v in mem}
        for v, g in owner.items():
            assert all(owner.get(u, g) == g for u in adj[v])
        assert all(v in owner or any(u in owner for u in adj[v]) for v in range(a.p))
        pos = {v: k for k, v in enumerate(order)} if order else {v: v for v in range(a.p)}
        for mem in got:
            opener = min(mem, key=lambda v: pos[v])
            assert all(v == opener or v in adj[opener] for v in mem)
            rows = int(sum(sizes[v] for v in mem))
            assert rows <= gmax or len(mem) == 1
            merged += len(mem) > 1
        info = o.level_info(lvl)
        assert info["nis"] == len(got) and info["n_is"] == sum(int(sizes[v]) for g in got for v in g)
    assert merged > 0


def test_group_zero_is_the_singleton_set(orc):
    s, og = _group_oracle(orc, "grid", 2, 1e-3, 0)
    s2, o1 = _group_oracle(orc, "grid", 2, 1e-3, 0)
    for lvl in range(og.nlevels):
        assert all(len(g) == 1 for g in _groups_of(og, lvl))
    x = np.random.default_rng(0).standard_normal(s.n)
    np.testing.assert_array_equal(og.apply(x), o1.apply(x))


def _group_rows(As, groups):
    ri = [np.arange(As.rb[v], As.rb[v + 1]) for g in groups for v in g]
    return np.concatenate(ri).astype(int) if ri else np.zeros(0, int)


@pytest.mark.parametrize("gmax", [8, 20])
@pytest.mark.parametrize("maker", ["grid", "random"])
def test_group_zero_drop_factorization_identity(orc, maker, gmax):
    """Eq. vbarms with groups at t = 0: [D F; E C] = [P^T L 0; W I] [U G; 0 S] with D block
    diagonal over the groups, and S the exact Schur complement."""
    s, o = _group_oracle(orc, maker, 1, 0.0, gmax)
    assert o.status == 0
    As = o.matrix(orc.AS, 0)
    a = As.dense()
    groups = _groups_of(o, 0)
    assert max(len(g) for g in groups) > 1
    ri = _group_rows(As, groups)
    inset = {v for g in groups for v in g}
    rr = np.concatenate([np.arange(As.rb[v], As.rb[v + 1]) for v in range(As.p) if v not in inset]).astype(int)
    D, F, E, Cm = a[np.ix_(ri, ri)], a[np.ix_(ri, rr)], a[np.ix_(rr, ri)], a[np.ix_(rr, rr)]
    S_exact = Cm - E @ np.linalg.solve(D, F)
    S = o.matrix(orc.LAST).dense()
    assert np.abs(S - S_exact).max() <= 1e-12 * np.abs(S_exact).max()
    dm = o.matrix(orc.D, 0)
    assert list(np.diff(dm.rb)) == [int(sum(np.diff(As.rb)[v] for v in g)) for g in groups]
    PtL, Uu = _block_lu_parts(dm)
    G = o.matrix(orc.G, 0).dense()
    Wm = o.matrix(orc.W, 0).dense()
    ni, nr = len(ri), len(rr)
    left = np.block([[PtL, np.zeros((ni, nr))], [Wm, np.eye(nr)]])
    right = np.block([[Uu, G], [np.zeros((nr, ni)), S]])
    full = np.block([[D, F], [E, Cm]])
    assert np.abs(left @ right - full).max() <= 1e-12 * np.abs(full).max()


@pytest.mark.parametrize("levels", [1, 2, 3])
@pytest.mark.parametrize("gmax", [10, 32])
def test_group_apply_is_exact_inverse_without_dropping(orc, levels, gmax):
    s, o = _group_oracle(orc, "upwind", levels, 0.0, gmax)
    assert o.status == 0
    x = np.random.default_rng(levels).standard_normal(s.n)
    ye = np.linalg.solve(s.dense(), x)
    assert np.abs(o.apply(x) - ye).max() <= 1e-10 * np.abs(ye).max()


def test_group_dropping_matches_dense_bruteforce(orc):
    """At 0 < t: a block of L^{-1}F is a group's rows against one remaining supernode and a
    block of E U^{-1} one remaining supernode against a whole group; each is kept iff its
    ||B||_F / (m n) >= t."""
    t = 0.01
    s, o = _group_oracle(orc, "grid", 1, [t, 0.0], 12)
    assert o.status == 0
    As = o.matrix(orc.AS, 0)
    a = As.dense()
    groups = _groups_of(o, 0)
    owner = {v: g for g, mem in enumerate(groups) for v in mem}
    rest = [v for v in range(As.p) if v not in owner]
    rnum = {v: k for k, v in enumerate(rest)}
    stored = {(i, int(As.colidx[k])) for i in range(As.p) for k in range(As.rowptr[i], As.rowptr[i + 1])}
    dm = o.matrix(orc.D, 0)
    PtL, Uu = _block_lu_parts(dm)
    rows = lambda v: np.arange(As.rb[v], As.rb[v + 1])
    Gx, Wx, margins = {}, {}, []
    for g, mem in enumerate(groups):
        rg = _group_rows(As, [mem])
        lo, hi = dm.rb[g], dm.rb[g + 1]
        for K in rest:
            if not any((v, K) in stored for v in mem):
                continue
            val = np.linalg.solve(PtL[lo:hi, lo:hi], a[np.ix_(rg, rows(K))])
            r = H.block_sumsq_ratio(val, t)
            margins.append(abs(r - 1))
            if r >= 1:
                Gx[(g, rnum[K])] = val
        for J in rest:
            if not any((J, v) in stored for v in mem):
                continue
            val = np.linalg.solve(Uu[lo:hi, lo:hi].T, a[np.ix_(rows(J), rg)].T).T
            r = H.block_sumsq_ratio(val, t)
            margins.append(abs(r - 1))
            if r >= 1:
                Wx[(rnum[J], g)] = val
    assert min(margins) > 1e-9

    def blocks(bm):
        return {(i, int(bm.colidx[k])): bm.block(k) for i in range(bm.p)
                for k in range(bm.rowptr[i], bm.rowptr[i + 1])}

    gb, wb = blocks(o.matrix(orc.G, 0)), blocks(o.matrix(orc.W, 0))
    assert set(gb) == set(Gx) and set(wb) == set(Wx)
    assert 0 < len(gb) < len(margins) and 0 < len(wb)
    for key in Gx:
        np.testing.assert_allclose(gb[key], Gx[key], rtol=1e-12, atol=1e-14)
    for key in Wx:
        np.testing.assert_allclose(wb[key], Wx[key], rtol=1e-12, atol=1e-14)


def test_groups_eliminate_more_rows_per_level(orc):
    s, og = _group_oracle(orc, "upwind", 1, 1e-3, 24)
    s, o1 = _group_oracle(orc, "upwind", 1, 1e-3, 0)
    assert og.level_info(0)["n_is"] > 1.25 * o1.level_info(0)["n_is"]


# --------------------------------------------------------------------------------------
# Last level block ILUT (Sec. 3, Alg. 3)
# --------------------------------------------------------------------------------------
def test_last_level_ilut_exact_without_dropping(orc):
    s = synth.grid_system(4, 4, 3, ell=3, stencil="14rand", perturb=0.1, seed=31)
    o, _, _ = _oracle(orc, s, 0.8, 1, 0.0)
    A = o.matrix(orc.LAST).dense()
    Lm = o.matrix(orc.L).dense() + np.eye(A.shape[0])
    Um = o.matrix(orc.U).dense()
    PtL, Uu = _block_lu_parts(o.matrix(orc.DL))
    Um = Um + PtL @ Uu
    assert np.abs(Lm @ Um - A).max() <= 1e-12 * np.abs(A).max()
    # block lower / upper structure
    Lb, Ub = o.matrix(orc.L), o.matrix(orc.U)
    for i in range(Lb.p):
        assert all(Lb.colidx[Lb.rowptr[i]:Lb.rowptr[i + 1]] < i)
        assert all(Ub.colidx[Ub.rowptr[i]:Ub.rowptr[i + 1]] > i)


def test_last_level_huge_threshold_is_block_jacobi(orc):
    s = synth.grid_system(3, 3, 3, ell=4, stencil="14rand", seed=32)
    o, _, _ = _oracle(orc, s, 1.0, 0, 1e9)
    assert o.matrix(orc.L).nb == 0 and o.matrix(orc.U).nb == 0
    A = o.matrix(orc.LAST)
    dl = o.matrix(orc.DL)
    for i in range(A.p):
        k = [kk for kk in range(A.rowptr[i], A.rowptr[i + 1]) if A.colidx[kk] == i][0]
        lu, piv = sla.lu_factor(A.block(k))
        np.testing.assert_allclose(dl.block(i), lu, rtol=1e-13, atol=1e-15)


def _blocks(bm):
    out = {}
    for i in range(bm.p):
        for k in range(bm.rowptr[i], bm.rowptr[i + 1]):
            out[(i, int(bm.colidx[k]))] = bm.block(k)
    return out


_ILUT_CASES = {
    # (system, levels, t): variable blocks of 1..7 unknowns; "shift" also forces row
    # interchanges inside every pivot block; levels = 1 runs the ILUT on a Schur complement
    "upwind-l0": (lambda: synth.upwind_system(4, 4, 3, seed=81), 0, 1e-2),
    "upwind-l1": (lambda: synth.upwind_system(4, 4, 3, seed=81), 1, 3e-3),
    "upwind-shift-l0": (lambda: H.node_rows_reversed(synth.upwind_system(4, 4, 3, seed=82), "shift"), 0, 1e-2),
    "upwind-shift-l1": (lambda: H.node_rows_reversed(synth.upwind_system(4, 4, 3, seed=82), "shift"), 1, 1e-2),
}


@pytest.mark.parametrize("case", sorted(_ILUT_CASES))
def test_last_level_ilut_dropping_matches_dense_bruteforce(orc, case):
    """Block ILUT at drop tolerances that keep some multipliers and U blocks and drop
    others (Sec. 3 drop rule inside Alg. 3): same kept sets and the same values as a dense
    block IKJ elimination written from the definition."""
    make, levels, t = _ILUT_CASES[case]
    s = make()
    o, _, _ = _oracle(orc, s, 1.0, levels, t)
    assert o.status == 0
    A = o.matrix(orc.LAST)
    if levels == 0:
        # with no reduction the ILUT input is the permuted input matrix itself
        perm, _ = orc.compress(s.n, s.rowptr, s.col, 1.0)
        np.testing.assert_array_equal(A.dense(), s.dense()[np.ix_(perm, perm)])
    Lb, Ub, Db, mr, ur = H.dense_block_ilut(A.dense(), A.rb, t)
    mr, ur = np.array(mr), np.array(ur)
    # both kinds of decision go both ways, and none is within rounding of the threshold
    assert np.sum(mr < 1) > 0 and np.sum(mr >= 1) > 0
    assert np.sum(ur < 1) > 0 and np.sum(ur >= 1) > 0
    assert np.min(np.abs(np.concatenate([mr, ur]) - 1.0)) > 1e-4
    # variable block sizes really occur (the drop threshold scales with m n)
    assert len(set(np.diff(A.rb).tolist())) > 3
    Lo, Uo = _blocks(o.matrix(orc.L)), _blocks(o.matrix(orc.U))
    assert set(Lo) == set(Lb)
    assert set(Uo) == set(Ub)
    for key, v in Lb.items():
        assert np.abs(Lo[key] - v).max() <= 1e-10 * np.abs(v).max()
    for key, v in Ub.items():
        assert np.abs(Uo[key] - v).max() <= 1e-10 * np.abs(v).max()
    PtL, Uu = _block_lu_parts(o.matrix(orc.DL))
    for i in range(A.p):
        a, b = A.rb[i], A.rb[i + 1]
        d = (PtL @ Uu)[a:b, a:b]
        assert np.abs(d - Db[i]).max() <= 1e-10 * np.abs(Db[i]).max()


# --------------------------------------------------------------------------------------
# Graph-based compression (Sec. 2.2, Alg. 1)
# --------------------------------------------------------------------------------------
def _no_diagonal_matrix(seed, n=40):
    """A random sparse pattern with no stored diagonal entry (rows couple only to others)."""
    rng = np.random.default_rng(650 + seed)
    pat = rng.random((n, n)) < 0.08
    np.fill_diagonal(pat, False)
    pat[np.arange(n), (np.arange(n) + 1) % n] = True
    rows, cols = np.nonzero(pat)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int64)
    return synth.System(n, rowptr, cols.astype(np.int32), rng.standard_normal(rows.size), np.zeros(n),
                        np.ones(n, np.int32), name=f"nodiag-{seed}")


_GRAPH_INPUTS = {
    "no_diagonal": _no_diagonal_matrix,
    "grid14": lambda seed: synth.grid_system(3, 3, 2, ell=3, stencil="14rand", perturb=0.15, seed=600 + seed),
    "random": lambda seed: synth.random_pattern_matrix(60, 0.05, twins=15, seed=610 + seed),
    "upwind": lambda seed: synth.upwind_system(3, 3, 2, perturb=0.1, seed=620 + seed),
}


@pytest.mark.parametrize("mu", [0.9, 0.7, 0.5])
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("kind", sorted(_GRAPH_INPUTS))
def test_graph_compression_matches_bruteforce(orc, kind, seed, mu):
    """Same partition as a set-based restatement of the greedy merging; every decision away
    from the threshold except exact ties, which both sides accept (nnz >= mu * elements)."""
    s = _GRAPH_INPUTS[kind](seed)
    perm, bptr = orc.graph_compress(s.n, s.rowptr, s.col, mu)
    p2, b2, margin = H.graph_compress_bruteforce(s.n, s.rowptr, s.col, mu)
    assert margin == 0.0 or margin > 1e-9
    np.testing.assert_array_equal(perm, p2)
    np.testing.assert_array_equal(bptr, b2)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_graph_compression_mu_one_keeps_identical_pattern_classes(orc, seed):
    s = synth.random_pattern_matrix(120, 0.04, twins=40, seed=630 + seed)
    perm, bptr = orc.graph_compress(s.n, s.rowptr, s.col, 1.0)
    p2, b2 = H.identical_pattern_partition(s.n, s.rowptr, s.col)
    np.testing.assert_array_equal(perm, p2)
    np.testing.assert_array_equal(bptr, b2)


@pytest.mark.parametrize("mu", [0.9, 0.7, 0.6])
def test_graph_compression_keeps_the_density_and_merges(orc, mu):
    """The average block density of the result is at least mu (the method's guarantee),
    blocks stay within 32 rows, and merging happened beyond the identical-pattern classes."""
    s = synth.grid_system(6, 5, 4, ell=4, stencil="14rand", perturb=0.15, seed=640)
    perm, bptr = orc.graph_compress(s.n, s.rowptr, s.col, mu)
    assert sorted(perm.tolist()) == list(range(s.n))
    assert H.average_block_density(s.n, s.rowptr, s.col, perm, bptr) >= mu
    assert np.diff(bptr).max() <= 32
    p1, b1 = H.identical_pattern_partition(s.n, s.rowptr, s.col)
    assert len(bptr) < len(b1)


# --------------------------------------------------------------------------------------
# Preconditioner application (Alg. 2)
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("levels", [0, 1, 2, 3])
def test_apply_is_exact_inverse_without_dropping(orc, levels):
    s = synth.grid_system(4, 3, 3, ell=3, stencil="14rand", perturb=0.1, seed=41)
    o, _, _ = _oracle(orc, s, 0.8, levels, 0.0)
    assert o.status == 0
    rng = np.random.default_rng(levels)
    x = rng.standard_normal(s.n)
    y = o.apply(x)
    ye = np.linalg.solve(s.dense(), x)
    assert np.abs(y - ye).max() <= 1e-10 * np.abs(ye).max()


def test_apply_with_dropping_is_linear_and_approximate(orc):
    s = synth.grid_system(5, 4, 4, ell=5, stencil="14rand", perturb=0.1, seed=42)
    o, _, _ = _oracle(orc, s, 0.8, 2, 1e-2)
    rng = np.random.default_rng(1)
    x1, x2 = rng.standard_normal(s.n), rng.standard_normal(s.n)
    y = o.apply(2.0 * x1 - 3.0 * x2)
    np.testing.assert_allclose(y, 2.0 * o.apply(x1) - 3.0 * o.apply(x2), rtol=1e-10, atol=1e-12)
    a = s.dense()
    err = np.linalg.norm(a @ o.apply(x1) - x1) / np.linalg.norm(x1)
    assert 1e-10 < err < 1.0


# --------------------------------------------------------------------------------------
# FGMRES (Sec. 4.1)
# --------------------------------------------------------------------------------------
def test_fgmres_unpreconditioned_history_is_krylov_least_squares(orc):
    rng = np.random.default_rng(3)
    n = 40
    a = np.eye(n) * 2.0 + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    rows, cols = np.nonzero(a)
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    x, st, its, rel, hist = orc.fgmres(n, rowptr, cols.astype(np.int32), a[rows, cols], b, None,
                                       tol=1e-15, restart=40, maxit=12)
    assert its == 12
    K = np.empty((n, 12))
    v = b.copy()
    for k in range(12):
        K[:, k] = v
        v = a @ v
    for k in range(1, 13):
        Q, _ = np.linalg.qr(K[:, :k])
        yk, *_ = np.linalg.lstsq(a @ Q, b, rcond=None)
        best = np.linalg.norm(b - a @ Q @ yk) / np.linalg.norm(b)
        assert abs(hist[k] - best) <= 1e-9 * max(best, 1e-12) + 1e-13
    assert np.all(np.diff(hist) <= 1e-15)


def test_fgmres_exact_preconditioner_converges_in_one_iteration(orc):
    s = synth.grid_system(4, 3, 3, ell=3, stencil="14rand", perturb=0.1, seed=51)
    o, _, _ = _oracle(orc, s, 0.8, 2, 0.0)
    x, st, its, rel, hist = orc.fgmres(s.n, s.rowptr, s.col, s.val, s.b, o, tol=1e-8, restart=30)
    assert st == 0 and its == 1 and rel <= 1e-8


def test_fgmres_true_residual_and_restarts(orc):
    s = synth.grid_system(6, 6, 6, ell=5, stencil="14rand", perturb=0.1, seed=52)
    o, _, _ = _oracle(orc, s, 0.8, 2, 5e-2)
    x, st, its, rel, hist = orc.fgmres(s.n, s.rowptr, s.col, s.val, s.b, o, tol=1e-8, restart=5)
    assert st == 0
    r = s.b - s.dense() @ x
    assert np.linalg.norm(r) / np.linalg.norm(s.b) <= 1e-8
    assert abs(np.linalg.norm(r) / np.linalg.norm(s.b) - rel) <= 1e-12
    assert its > 5  # needed at least one restart
    x, st, its, rel, hist = orc.fgmres(s.n, s.rowptr, s.col, s.val, s.b, o, tol=1e-8, restart=5, maxit=2)
    assert st == orc.NOT_CONVERGED and its == 2


def test_singular_pivot_block_reported(orc):
    s = synth.grid_system(3, 3, 2, ell=3, stencil="7pt", seed=61)
    val = s.val.copy()
    # zero out every entry of node 0's diagonal block -> its pivot block is singular
    for r in range(3):
        for k in range(s.rowptr[r], s.rowptr[r + 1]):
            if s.col[k] < 3:
                val[k] = 0.0
    perm, bptr = orc.compress(s.n, s.rowptr, s.col, 1.0)
    o = orc.Oracle(s.n, s.rowptr, s.col, val, perm, bptr, 1, 1e-3)
    assert o.status == orc.ERR_SINGULAR and o.err_level == 0 and o.err_block == 0


# --------------------------------------------------------------------------------------
# Inputs that force row pivoting inside every pivot block
# --------------------------------------------------------------------------------------
def _pivoting_system(mode="reverse"):
    return H.node_rows_reversed(synth.grid_system(4, 3, 3, ell=4, stencil="14rand", seed=71), mode)


def test_pivoting_pivot_blocks_match_lapack_getrf(orc):
    s = _pivoting_system()
    o, _, _ = _oracle(orc, s, 1.0, 1, 0.0)
    asd = o.matrix(orc.AS, 0)
    dm = o.matrix(orc.D, 0)
    swaps = 0
    for t, i in enumerate(o.level_is(0)):
        k = [kk for kk in range(asd.rowptr[i], asd.rowptr[i + 1]) if asd.colidx[kk] == i][0]
        lu, piv = sla.lu_factor(asd.block(k))
        got = dm.piv[dm.rb[t]:dm.rb[t + 1]]
        np.testing.assert_array_equal(got, piv)
        swaps += int(np.sum(got != np.arange(len(got))))
        np.testing.assert_allclose(dm.block(t), lu, rtol=1e-13, atol=1e-15)
    assert swaps > 0


@pytest.mark.parametrize("mode", ["reverse", "shift"])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_pivoting_apply_is_exact_inverse(orc, levels, mode):
    s = _pivoting_system(mode)
    o, _, _ = _oracle(orc, s, 1.0, levels, 0.0)
    assert o.status == 0
    x = np.random.default_rng(7).standard_normal(s.n)
    ye = np.linalg.solve(s.dense(), x)
    y = o.apply(x)
    assert np.abs(y - ye).max() <= 1e-10 * np.abs(ye).max()


@pytest.mark.parametrize("mode", ["reverse", "shift"])
def test_pivoting_zero_drop_identity_and_ilut(orc, mode):
    s = _pivoting_system(mode)
    o, _, _ = _oracle(orc, s, 1.0, 1, 0.0)
    As = o.matrix(orc.AS, 0)
    a = As.dense()
    ri, rr = _split(As, o.level_is(0))
    D, F, E, Cm = a[np.ix_(ri, ri)], a[np.ix_(ri, rr)], a[np.ix_(rr, ri)], a[np.ix_(rr, rr)]
    PtL, Uu = _block_lu_parts(o.matrix(orc.D, 0))
    G = o.matrix(orc.G, 0).dense()
    Wm = o.matrix(orc.W, 0).dense()
    np.testing.assert_allclose(PtL @ G, F, atol=1e-12 * np.abs(F).max())
    np.testing.assert_allclose(Wm @ Uu, E, atol=1e-12 * np.abs(E).max())
    S = o.matrix(orc.LAST).dense()
    S_exact = Cm - E @ np.linalg.solve(D, F)
    assert np.abs(S - S_exact).max() <= 1e-12 * np.abs(S_exact).max()
    Lm = o.matrix(orc.L).dense() + np.eye(S.shape[0])
    PtL2, Uu2 = _block_lu_parts(o.matrix(orc.DL))
    Um = o.matrix(orc.U).dense() + PtL2 @ Uu2
    assert np.abs(Lm @ Um - S).max() <= 1e-12 * np.abs(S).max()
    # the multipliers are L_ik = w_k D_k^{-1}: check one against a dense solve
    Lb = o.matrix(orc.L)
    assert Lb.nb > 0


# --------------------------------------------------------------------------------------
# Inputs on which the first GPU version faulted (kept off the GPU): valid on the CPU
# --------------------------------------------------------------------------------------
def _panel_layout_in_bounds(bm):
    """Restates the panel layout of a block matrix (row widths, value offsets, block column
    offsets, scalar columns) and checks every index it produces against its array."""
    rs, cs = np.diff(bm.rb), np.diff(bm.cb)
    assert rs.max(initial=0) <= 32 and cs.max(initial=0) <= 32
    nv = 0
    n_cols = int(bm.cb[-1])
    for i in range(bm.p):
        ks = range(bm.rowptr[i], bm.rowptr[i + 1])
        cols = [int(bm.colidx[k]) for k in ks]
        assert cols == sorted(set(cols)) and all(0 <= c < bm.q for c in cols)
        width = int(sum(cs[c] for c in cols))
        co = np.concatenate([[0], np.cumsum([cs[c] for c in cols])])[:-1] if cols else np.zeros(0, int)
        for c, o in zip(cols, co):
            assert o + cs[c] <= width
            sc = np.arange(bm.cb[c], bm.cb[c + 1])
            assert sc.min() >= 0 and sc.max() < n_cols
        nv += int(rs[i]) * width
    assert nv == int(bm.voff[-1])


@pytest.mark.parametrize("case", ["smoke_8x8x6", "tiny_2x2x1_seed0", "tiny_2x2x1_seed1", "tiny_2x2x1_seed2"])
def test_inputs_that_faulted_the_first_gpu_version_are_valid_on_the_cpu(orc, case):
    """The smoke input (8x8x6 14-neighbour grid, ell = 5, tau = 0.8, 3 levels, t = 1e-4) and a
    2x2x1 7-point grid (ell = 2, tau = 1, levels = 0, t = 0) ended the first GPU version with
    a memory fault; they stay off the GPU.  On the CPU every intermediate is well formed:
    the partition is a permutation into blocks of at most 32 rows, every level matrix and
    factor has a panel layout whose indices stay inside its arrays, and the factorization is
    what the method prescribes (the exact inverse at t = 0)."""
    if case == "smoke_8x8x6":
        s = synth.grid_system(8, 8, 6, ell=5, stencil="14rand", perturb=0.10, seed=2)
        tau, levels, t = 0.8, 3, 1e-4
    else:
        s = synth.grid_system(2, 2, 1, ell=2, stencil="7pt", seed=int(case[-1]))
        tau, levels, t = 1.0, 0, 0.0
    o, perm, bptr = _oracle(orc, s, tau, levels, t)
    assert o.status == 0
    assert sorted(perm.tolist()) == list(range(s.n))
    assert bptr[0] == 0 and bptr[-1] == s.n and np.all(np.diff(bptr) >= 1) and np.diff(bptr).max() <= 32
    for lvl in range(o.nlevels):
        for w in (orc.A, orc.AS, orc.G, orc.W):
            _panel_layout_in_bounds(o.matrix(w, lvl))
    for w in (orc.LAST, orc.L, orc.U):
        _panel_layout_in_bounds(o.matrix(w))
    if t == 0.0:
        x = np.random.default_rng(0).standard_normal(s.n)
        ye = np.linalg.solve(s.dense(), x)
        assert np.abs(o.apply(x) - ye).max() <= 1e-10 * np.abs(ye).max()
