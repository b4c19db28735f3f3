"""Seeded synthetic inputs shaped like the paper's block-structured Navier-Stokes Jacobians.

This module only produces inputs (a CSR matrix, a right-hand side and the node
layout). It performs none of the preconditioner's arithmetic, so both the GPU path
and the CPU oracle can be driven from it.

Shapes follow the RANS application of Sec. 4.2: ell unknowns per mesh node
(ell = 5 for incompressible RANS with one turbulence equation), a symmetric node
graph with about 7 neighbour blocks per row in 2D and 14 in 3D, and nonsymmetric
values (Sec. 4.2, discussion after the implicit-scheme equation).

Recipes
-------
* ``grid7``: nx*ny*nz nodes, 7-point stencil, lexicographic node numbering,
  unknowns numbered node-major.  A_uu = N(0,1) + 8 I;
  A_uv = -0.5 I + 0.3 (v_u . n_uv) N(0,1), v_u ~ U(-1,1)^3, n_uv the unit offset.
* ``grid14``: the 6 face links plus each of the 20 edge/corner links kept with
  probability 0.4; the keep decision is a hash of (seed, min(u,v), max(u,v)) so the
  node graph is symmetric.  Same values as ``grid7``.  Optionally every entry of
  every block is perturbed with probability ``perturb``: half of those are removed
  from the pattern, half are scaled by 1e-6.  Point-diagonal entries are never
  perturbed.
* ``upwind``: per-node block size ell_u drawn from a list, cell Peclet number
  Pe_u ~ LogUniform, unit velocity direction d_u;
  w_uv = (1 + Pe_u max(0, -d_u . n_uv)) / 14,
  A_uv = -w_uv I_rect + 0.3 w_uv N(0,1),  A_uu = (1 + sum_v w_uv) I + 0.3 N(0,1).
"""
from __future__ import annotations

import dataclasses
import numpy as np

__all__ = ["System", "grid_system", "upwind_system", "random_pattern_matrix", "dense_rows_matrix", "config_system"]

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


@dataclasses.dataclass
class System:
    """A sparse system in CSR form (int64 rowptr, int32 col sorted per row, float64 val)."""

    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray
    node_ell: np.ndarray  # block size per node, in node order
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        for i in range(self.n):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            a[i, self.col[s:e]] = self.val[s:e]
        return a


def _splitmix(x: np.ndarray) -> np.ndarray:
    x = (x + np.uint64(0x9E3779B97F4A7C15)) & _M64
    x = ((x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
    x = ((x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
    return x ^ (x >> np.uint64(31))


def _link_keep(seed: int, u: np.ndarray, v: np.ndarray, prob: float) -> np.ndarray:
    lo = np.minimum(u, v).astype(np.uint64)
    hi = np.maximum(u, v).astype(np.uint64)
    with np.errstate(over="ignore"):
        h = _splitmix(np.uint64(seed) * np.uint64(0x100000001B3) ^ _splitmix(lo * np.uint64(0x2545F4914F6CDD1D) ^ hi))
    return (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0) < prob


def _node_links(nx: int, ny: int, nz: int, stencil: str, seed: int):
    """Directed node links (u, v, unit offset) sorted by (u, v); symmetric by construction."""
    nodes = nx * ny * nz
    idx = np.arange(nodes, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    offs = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                k = abs(dx) + abs(dy) + abs(dz)
                if k == 0:
                    continue
                if stencil == "7pt" and k != 1:
                    continue
                offs.append((dx, dy, dz, k))
    us, vs, ns = [], [], []
    for dx, dy, dz, k in offs:
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
        u = idx[ok]
        v = u + dx + nx * dy + nx * ny * dz
        if k > 1:
            keep = _link_keep(seed, u, v, 0.4)
            u, v = u[keep], v[keep]
        nrm = np.array([dx, dy, dz], dtype=np.float64) / np.sqrt(k)
        us.append(u)
        vs.append(v)
        ns.append(np.broadcast_to(nrm, (u.size, 3)))
    u = np.concatenate(us)
    v = np.concatenate(vs)
    nvec = np.concatenate(ns)
    order = np.lexsort((v, u))
    return nodes, u[order], v[order], nvec[order]


def _csr_from_coo(n, rows, cols, vals):
    # row-major order of the entries (a stable sort on one key: the same order as sorting
    # by row, then column, then position)
    o = np.argsort(np.asarray(rows, np.int64) * np.int64(n) + np.asarray(cols, np.int64), kind="stable")
    rows, cols, vals = rows[o], cols[o], vals[o]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    np.cumsum(rowptr, out=rowptr)
    return rowptr, cols.astype(np.int32), vals.astype(np.float64)


def _rhs(n, rowptr, val, b_kind, rng):
    if b_kind == "ones":
        # b = A * ones, i.e. the row sums
        b = np.zeros(n)
        nz = np.diff(rowptr) > 0
        sums = np.add.reduceat(val, rowptr[:-1][nz]) if val.size else np.zeros(0)
        b[nz] = sums
        return b
    return rng.standard_normal(n)


def grid_system(nx: int, ny: int, nz: int, ell: int = 5, stencil: str = "7pt", perturb: float = 0.0,
                seed: int = 1, b_kind: str = "ones") -> System:
    """The ``grid7`` / ``grid14`` recipes with a uniform block size ``ell``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    st = "7pt" if stencil == "7pt" else "14rand"
    nodes, u, v, nvec = _node_links(nx, ny, nz, st, seed)
    vel = rng.uniform(-1.0, 1.0, size=(nodes, 3))
    e = ell
    diag = rng.standard_normal((nodes, e, e)) + 8.0 * np.eye(e)
    coef = 0.3 * np.einsum("ij,ij->i", vel[u], nvec)
    off = -0.5 * np.eye(e)[None, :, :] + coef[:, None, None] * rng.standard_normal((u.size, e, e))
    # vectorised assembly: every node block is e x e
    all_u = np.concatenate([np.arange(nodes), u])
    all_v = np.concatenate([np.arange(nodes), v])
    blocks = np.concatenate([diag, off], axis=0)
    r_loc = np.repeat(np.arange(e), e)
    c_loc = np.tile(np.arange(e), e)
    rows = (all_u[:, None] * e + r_loc[None, :]).ravel()
    cols = (all_v[:, None] * e + c_loc[None, :]).ravel()
    vals = blocks.reshape(-1)
    n = nodes * e
    if perturb > 0.0:
        hit = rng.random(vals.size) < perturb
        remove = rng.random(vals.size) < 0.5
        point_diag = rows == cols
        hit &= ~point_diag
        vals = np.where(hit & ~remove, vals * 1e-6, vals)
        keep = ~(hit & remove)
        rows, cols, vals = rows[keep], cols[keep], vals[keep]
    rowptr, col, val = _csr_from_coo(n, rows, cols, vals)
    b = _rhs(n, rowptr, val, b_kind, rng)
    return System(n, rowptr, col, val, b, np.full(nodes, e, dtype=np.int32),
                  name=f"{st}-{nx}x{ny}x{nz}-l{e}-p{perturb}-s{seed}")


def upwind_system(nx: int, ny: int, nz: int, ell_choices=(1, 2, 3, 4, 5, 6, 7), pe_range=(0.1, 100.0),
                  stencil: str = "14rand", anisotropy: float = 1.0, perturb: float = 0.0, seed: int = 3,
                  b_kind: str = "ones") -> System:
    """The ``upwind`` recipe: variable block sizes and convection-driven nonsymmetry."""
    rng = np.random.Generator(np.random.PCG64(seed))
    st = "7pt" if stencil == "7pt" else "14rand"
    nodes, u, v, nvec = _node_links(nx, ny, nz, st, seed)
    ell = rng.choice(np.asarray(ell_choices, dtype=np.int64), size=nodes)
    lo, hi = np.log(pe_range[0]), np.log(pe_range[1])
    pe = np.exp(rng.uniform(lo, hi, size=nodes))
    d = rng.standard_normal((nodes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    w = (1.0 + pe[u] * np.maximum(0.0, -np.einsum("ij,ij->i", d[u], nvec))) / 14.0
    if anisotropy != 1.0:
        w = np.where(np.abs(nvec[:, 2]) > 0, w * anisotropy, w)
    wsum = np.zeros(nodes)
    np.add.at(wsum, u, w)
    start = np.zeros(nodes + 1, dtype=np.int64)
    np.cumsum(ell, out=start[1:])
    n = int(start[-1])
    rows_l, cols_l, vals_l = [], [], []
    # group blocks by (ell_u, ell_v) so each group is drawn and placed vectorised
    all_u = np.concatenate([np.arange(nodes), u])
    all_v = np.concatenate([np.arange(nodes), v])
    is_diag = np.concatenate([np.ones(nodes, bool), np.zeros(u.size, bool)])
    all_w = np.concatenate([1.0 + wsum, w])
    eu, ev = ell[all_u], ell[all_v]
    for a in np.unique(eu):
        for bb in np.unique(ev):
            sel = np.nonzero((eu == a) & (ev == bb))[0]
            if sel.size == 0:
                continue
            eye = np.eye(a, bb)
            g = rng.standard_normal((sel.size, a, bb))
            sgn = np.where(is_diag[sel], 1.0, -1.0)
            blk = (sgn * all_w[sel])[:, None, None] * eye[None] + 0.3 * np.where(
                is_diag[sel], 1.0, all_w[sel])[:, None, None] * g
            rl = np.repeat(np.arange(a), bb)
            cl = np.tile(np.arange(bb), a)
            rows_l.append((start[all_u[sel]][:, None] + rl[None, :]).ravel())
            cols_l.append((start[all_v[sel]][:, None] + cl[None, :]).ravel())
            vals_l.append(blk.reshape(-1))
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    vals = np.concatenate(vals_l)
    if perturb > 0.0:
        hit = rng.random(vals.size) < perturb
        remove = rng.random(vals.size) < 0.5
        hit &= rows != cols
        vals = np.where(hit & ~remove, vals * 1e-6, vals)
        keep = ~(hit & remove)
        rows, cols, vals = rows[keep], cols[keep], vals[keep]
    rowptr, col, val = _csr_from_coo(n, rows, cols, vals)
    b = _rhs(n, rowptr, val, b_kind, rng)
    return System(n, rowptr, col, val, b, ell.astype(np.int32),
                  name=f"upwind-{nx}x{ny}x{nz}-s{seed}")


def random_pattern_matrix(n: int, density: float, twins: int = 0, seed: int = 0, diag: float = 4.0) -> System:
    """Small random sparse matrix with a nonzero diagonal and optional groups of identical rows.

    ``twins`` rows are made copies of the pattern of a randomly chosen earlier row
    (values are drawn independently), so exact-pattern classes exist.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    pat = rng.random((n, n)) < density
    np.fill_diagonal(pat, True)
    for _ in range(twins):
        i, j = rng.choice(n, size=2, replace=False)
        pat[i, j] = True  # both rows then hold both diagonal positions
        pat[j] = pat[i]
    a = np.where(pat, rng.standard_normal((n, n)), 0.0)
    a[pat & (a == 0.0)] = 1.0
    a += diag * np.eye(n) * pat.diagonal()
    rows, cols = np.nonzero(pat)
    vals = a[rows, cols]
    rowptr, col, val = _csr_from_coo(n, rows, cols, vals)
    b = _rhs(n, rowptr, val, "ones", rng)
    return System(n, rowptr, col, val, b, np.ones(n, np.int32), name=f"rand-{n}-{density}-s{seed}")


def dense_rows_matrix(n: int, row_len: int = 5, n_dense: int = 4, dense_len: int = 1200, core: int = 1000,
                      seed: int = 0) -> System:
    """Sparse random rows plus a few long rows that share a common core of columns.

    Each ordinary row holds its diagonal and ``row_len`` random columns; each long row holds
    its diagonal, the ``core`` shared columns and random ones up to ``dense_len``.  A long
    row then meets thousands of other rows through its columns (two-hop neighbours), and
    the long rows resemble each other (cosine about core / dense_len)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rows_l, cols_l = [], []
    for i in range(n):
        c = rng.choice(n, size=row_len, replace=False)
        rows_l.append(np.full(row_len + 1, i))
        cols_l.append(np.concatenate([[i], c]))
    dense = rng.choice(n, size=n_dense, replace=False)
    shared = rng.choice(n, size=core, replace=False)
    for i in dense:
        extra = rng.choice(n, size=dense_len - core, replace=False)
        c = np.unique(np.concatenate([[i], shared, extra]))
        rows_l.append(np.full(c.size, i))
        cols_l.append(c)
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    key = np.unique(rows.astype(np.int64) * n + cols)
    rows, cols = key // n, key % n
    vals = rng.standard_normal(rows.size)
    vals = np.where(rows == cols, 10.0 + np.abs(vals), vals)
    rowptr, col, val = _csr_from_coo(n, rows, cols, vals)
    b = _rhs(n, rowptr, val, "ones", rng)
    return System(n, rowptr, col, val, b, np.ones(n, np.int32), name=f"denserows-{n}-{n_dense}x{dense_len}-s{seed}")


def config_system(index: int, scale: float = 1.0) -> System:
    """Synthetic stand-ins for the benchmark configurations (1-based index).

    1: 10^3 grid, 7-point, ell=5, b = A 1.
    2: 40^3 grid, 14-neighbour random stencil, ell=5, 10% block-entry perturbation.
    3: 74^3 nodes, 14-neighbour stencil, ell ~ U{1..7}, upwind values.
    ``scale`` shrinks the grid side (for tests), keeping the recipe.
    """
    if index == 1:
        s = max(2, int(round(10 * scale)))
        return grid_system(s, s, s, 5, "7pt", 0.0, seed=1)
    if index == 2:
        s = max(2, int(round(40 * scale)))
        return grid_system(s, s, s, 5, "14rand", 0.10, seed=2)
    if index == 3:
        s = max(2, int(round(74 * scale)))
        return upwind_system(s, s, s, seed=3)
    raise ValueError(f"unknown configuration {index}")
