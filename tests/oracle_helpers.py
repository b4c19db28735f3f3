"""Brute-force references used to pin the CPU oracle (dense NumPy, tiny inputs)."""
from __future__ import annotations

import numpy as np


def patterns(n, rowptr, col):
    return [tuple(col[rowptr[i]:rowptr[i + 1]].tolist()) for i in range(n)]


def identical_pattern_partition(n, rowptr, col):
    """Groups of rows with the same nonempty pattern, ordered by smallest member; empty rows alone."""
    first = {}
    group = np.empty(n, dtype=np.int64)
    for i, pat in enumerate(patterns(n, rowptr, col)):
        if len(pat) == 0:
            group[i] = i
            continue
        group[i] = first.setdefault(pat, i)
    return _partition_from_group(group)


def _partition_from_group(group):
    n = len(group)
    seeds = sorted(set(group.tolist()))
    perm, bptr = [], [0]
    for s in seeds:
        members = [i for i in range(n) if group[i] == s]
        perm.extend(members)
        bptr.append(len(perm))
    return np.array(perm, dtype=np.int32), np.array(bptr, dtype=np.int32)


def angle_partition_bruteforce(n, rowptr, col, tau):
    """Sequential seed loop with cosines from the dense pattern product C C^T (float, with sqrt).

    Returns (perm, bptr, closest_margin) where closest_margin is the smallest |cos - tau|
    seen, so callers can make sure no decision was borderline."""
    c = np.zeros((n, n))
    for i in range(n):
        c[i, col[rowptr[i]:rowptr[i + 1]]] = 1.0
    g = c @ c.T
    ln = np.diag(g).copy()
    group = -np.ones(n, dtype=np.int64)
    margin = np.inf
    for i in range(n):
        if group[i] != -1:
            continue
        group[i] = i
        if ln[i] == 0:
            continue
        for j in range(i + 1, n):
            if group[j] != -1 or ln[j] == 0:
                continue
            cos = g[i, j] / np.sqrt(ln[i] * ln[j])
            margin = min(margin, abs(cos - tau))
            if cos >= tau:
                group[j] = i
    perm, bptr = _partition_from_group(group)
    return perm, bptr, margin


def greedy_is_bruteforce(adj_sets):
    """Natural-order greedy independent set on an undirected graph given as neighbour sets."""
    p = len(adj_sets)
    marked = np.zeros(p, bool)
    out = []
    for v in range(p):
        if marked[v]:
            continue
        out.append(v)
        marked[v] = True
        for u in adj_sets[v]:
            marked[u] = True
    return np.array(out, dtype=np.int32)


def quotient_adjacency(bm):
    """Neighbour sets of the quotient graph of A + A^T from a block matrix (self loops removed)."""
    adj = [set() for _ in range(bm.p)]
    for i in range(bm.p):
        for k in range(bm.rowptr[i], bm.rowptr[i + 1]):
            j = int(bm.colidx[k])
            if j != i:
                adj[i].add(j)
                adj[j].add(i)
    return adj


def block_sumsq_ratio(b, t):
    m, n = b.shape
    return float(np.sum(b * b)) / (t * m * n) ** 2


def node_rows_reversed(s, mode="reverse"):
    """The system with the rows of every node block reversed (or cyclically shifted by one).

    The block pattern is unchanged, but each diagonal block's dominant entries move off
    its diagonal, so partial pivoting has to swap rows in every pivot block; the cyclic
    shift makes successive swaps share rows, so their order matters."""
    from paper_1508_02219_amd.synth import System
    ell = np.asarray(s.node_ell, dtype=np.int64)
    start = np.concatenate([[0], np.cumsum(ell)])
    newrow = np.empty(s.n, dtype=np.int64)
    for u in range(len(ell)):
        a, b = start[u], start[u + 1]
        if mode == "reverse":
            newrow[a:b] = np.arange(b - 1, a - 1, -1)
        else:
            newrow[a:b] = a + (np.arange(b - a) - 1) % (b - a)
    order = np.argsort(newrow)  # new row r takes old row order[r]
    counts = np.diff(s.rowptr)[order]
    rowptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    col = np.concatenate([s.col[s.rowptr[o]:s.rowptr[o + 1]] for o in order]).astype(np.int32)
    val = np.concatenate([s.val[s.rowptr[o]:s.rowptr[o + 1]] for o in order])
    return System(s.n, rowptr, col, val, s.b[order], s.node_ell, name=s.name + "-rev")


def dense_block_ilut(a, rb, t):
    """Block IKJ ILUT with threshold t on a dense matrix (Alg. 3 read blockwise, Sec. 3).

    Written from the algorithm's definition, with none of the oracle's structure: row i is
    the dense block row w = A_i,: ; for k = 0 .. i-1 in ascending order the multiplier
    w_k D_k^{-1} is formed with a dense inverse of row k's (unfactored) diagonal block and
    dropped when ||w_k||_F / (m m_k) < t, otherwise every w_j, j > k, loses w_k U_kj.
    Blocks that are structurally absent are zero here, and a zero multiplier is always
    dropped for t > 0, so they change nothing.  Then U_ii = w_i and the blocks w_j, j > i,
    that pass the same test (kept when not below t) form U row i.

    Returns (L, U, D, mult_ratios, u_ratios): dicts (i, k) -> multiplier, (i, j) -> U
    block, i -> U_ii before factorization, and the ratios ||B||_F^2 / (t m n)^2 of every
    drop decision taken on a nonzero multiplier and on a nonzero off-diagonal U candidate
    (a ratio below 1 drops the block; callers check the margins)."""
    p = len(rb) - 1
    L, U, D = {}, {}, {}
    mult_ratios, u_ratios = [], []

    def blk(w, j):
        return w[:, rb[j]:rb[j + 1]]

    for i in range(p):
        w = a[rb[i]:rb[i + 1], :].copy()
        m = rb[i + 1] - rb[i]
        for k in range(i):
            wk = blk(w, k)
            if not np.any(wk):
                continue
            mult = wk @ np.linalg.inv(D[k])
            mk = rb[k + 1] - rb[k]
            r = float(np.sum(mult * mult)) / (t * m * mk) ** 2
            mult_ratios.append(r)
            wk[:, :] = 0.0
            if r < 1.0:
                continue
            L[(i, k)] = mult
            for j in range(k + 1, p):
                if (k, j) in U:
                    w[:, rb[j]:rb[j + 1]] -= mult @ U[(k, j)]
        D[i] = blk(w, i).copy()
        for j in range(i + 1, p):
            wj = blk(w, j)
            if not np.any(wj):
                continue
            r = float(np.sum(wj * wj)) / (t * m * (rb[j + 1] - rb[j])) ** 2
            u_ratios.append(r)
            if r >= 1.0:
                U[(i, j)] = wj.copy()
    return L, U, D, mult_ratios, u_ratios


def graph_compress_bruteforce(n, rowptr, col, mu, max_block=32):
    """Greedy merging of supernodes (Sec. 2.2, Alg. 1) written with Python sets: start from the
    identical-pattern classes; for every supernode in ascending smallest row, try its
    quotient-graph neighbours (A + A^T) in ascending smallest row and keep a merge when the
    average block density of the whole ordering stays >= mu.  Returns (perm, bptr,
    closest_margin), the margin being the smallest |nnz - mu * elements| / nnz seen."""
    pats = [tuple(col[rowptr[i]:rowptr[i + 1]].tolist()) for i in range(n)]
    first = {}
    label = [first.setdefault(pats[i], i) for i in range(n)]
    members = {}
    for i in range(n):
        members.setdefault(label[i], set()).add(i)
    entries = [(i, int(j)) for i in range(n) for j in col[rowptr[i]:rowptr[i + 1]]]
    nnz = len(entries)
    nbr = [set() for _ in range(n)]
    for i, j in entries:
        nbr[i].add(j)
        nbr[j].add(i)

    def elements(lab, mem):
        blocks = {(lab[i], lab[j]) for i, j in entries} | {(s, s) for s in mem}
        return sum(len(mem[a]) * len(mem[b]) for a, b in blocks)

    margin = float("inf")
    for X in sorted(members):
        if X not in members:
            continue
        cand = sorted({label[j] for i in members[X] for j in nbr[i]} - {X}, key=lambda s: min(members[s]))
        for Z in cand:
            if Z not in members or len(members[X]) + len(members[Z]) > max_block:
                continue
            lab2 = [X if label[i] == Z else label[i] for i in range(n)]
            mem2 = {k: v for k, v in members.items() if k != Z}
            mem2[X] = members[X] | members[Z]
            el = elements(lab2, mem2)
            margin = min(margin, abs(nnz - mu * el) / nnz)
            if nnz >= mu * el:
                label, members = lab2, mem2
    blocks = sorted(members.values(), key=min)
    perm = [i for b in blocks for i in sorted(b)]
    bptr = np.concatenate([[0], np.cumsum([len(b) for b in blocks])])
    return np.array(perm, np.int32), bptr.astype(np.int32), margin


def average_block_density(n, rowptr, col, perm, bptr):
    """nnz / elements of the blocks holding an entry or on the diagonal, for a partition."""
    blk = np.empty(n, np.int64)
    for b in range(len(bptr) - 1):
        blk[perm[bptr[b]:bptr[b + 1]]] = b
    sizes = np.diff(bptr)
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    pairs = set(zip(blk[rows].tolist(), blk[np.asarray(col)].tolist())) | {(b, b) for b in range(len(sizes))}
    return len(col) / float(sum(int(sizes[a]) * int(sizes[b]) for a, b in pairs))


def greedy_groups_bruteforce(adj_sets, sizes, gmax, order=None):
    """Greedy block independent set with groups of nodes on an undirected graph: an
    unmarked vertex v opens a group, its unmarked neighbours join in ascending order when
    the group stays within gmax rows, then the group and its neighbourhood are marked.
    Returns the groups (members ascending) ordered by their smallest member."""
    p = len(adj_sets)
    marked = [False] * p
    groups = []
    for v in (range(p) if order is None else order):
        if marked[v]:
            continue
        mem = [v]
        marked[v] = True
        rows = int(sizes[v])
        for u in sorted(adj_sets[v]):
            if not marked[u] and rows + int(sizes[u]) <= gmax:
                mem.append(u)
                marked[u] = True
                rows += int(sizes[u])
        for w in mem:
            for u in adj_sets[w]:
                marked[u] = True
        groups.append(sorted(mem))
    return sorted(groups, key=lambda g: g[0])
