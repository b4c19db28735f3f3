"""ctypes wrapper of the VBARMS CPU oracle (vbarms_oracle.c) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It never touches the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vbarms_oracle.c")
LIB = os.environ.get("VBARMS_ORACLE_LIB") or os.path.join(HERE, "liborc.so")

OK, NOT_CONVERGED, ERR_ARG, ERR_OOM, ERR_SINGULAR, ERR_STATE = 0, 1, -1, -3, -4, -6
# matrices that can be exported
A, AS, G, W, D, LAST, L, U, DL = range(9)

_lib = None


def build(force: bool = True, src: str = SRC, out: str | None = None) -> str:
    """Compile the oracle with gcc (no fused multiply-add, plain -O2)."""
    out = out or LIB
    if force or not os.path.exists(out):
        tmp = out + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        l = C.CDLL(LIB)
        P = C.c_void_p
        i32, i64, dbl = C.c_int32, C.c_int64, C.c_double
        l.orc_compress.argtypes = [C.c_int, P, P, dbl, P, P, P]
        l.orc_compress.restype = C.c_int
        l.orc_graph_compress.argtypes = [C.c_int, P, P, dbl, P, P, P]
        l.orc_graph_compress.restype = C.c_int
        l.orc_build.argtypes = [C.c_int, P, P, P, P, P, C.c_int, C.c_int, P, C.c_int, C.c_int, C.c_int]
        l.orc_build.restype = P
        l.orc_free.argtypes = [P]
        l.orc_status.argtypes = [P, P, P]
        l.orc_status.restype = C.c_int
        l.orc_apply.argtypes = [P, P, P]
        l.orc_apply.restype = C.c_int
        l.orc_fgmres.argtypes = [P, C.c_int, P, P, P, P, P, dbl, C.c_int, C.c_int, P, P, P]
        l.orc_fgmres.restype = C.c_int
        l.orc_nlevels.argtypes = [P]
        l.orc_nlevels.restype = C.c_int
        l.orc_level_info.argtypes = [P, C.c_int, P]
        l.orc_level_is.argtypes = [P, C.c_int, P]
        l.orc_level_groups.argtypes = [P, C.c_int, P]
        l.orc_level_scaling.argtypes = [P, C.c_int, P, P]
        l.orc_matrix_dims.argtypes = [P, C.c_int, C.c_int, P]
        l.orc_matrix_dims.restype = C.c_int
        l.orc_matrix_get.argtypes = [P, C.c_int, C.c_int, P, P, P, P, P, P]
        l.orc_matrix_get.restype = C.c_int
        l.orc_factor_nnz.argtypes = [P]
        l.orc_factor_nnz.restype = i64
        _lib = l
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _csr(rowptr, col, val=None):
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    v = None if val is None else np.ascontiguousarray(val, dtype=np.float64)
    return rp, ci, v


def compress(n, rowptr, col, tau):
    """Angle-based compression (Sec. 2.1). Returns (perm, bptr)."""
    rp, ci, _ = _csr(rowptr, col)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    bptr = np.zeros(n + 1, dtype=np.int32)
    p = np.zeros(1, dtype=np.int32)
    st = lib().orc_compress(n, _p(rp), _p(ci), float(tau), _p(perm), _p(bptr), _p(p))
    if st != OK:
        raise ValueError(f"orc_compress failed ({st})")
    return perm[:n].copy(), bptr[: p[0] + 1].copy()


def graph_compress(n, rowptr, col, mu):
    """Graph-based compression with target density mu (Sec. 2.2, Alg. 1). Returns (perm, bptr)."""
    rp, ci, _ = _csr(rowptr, col)
    perm = np.zeros(max(n, 1), dtype=np.int32)
    bptr = np.zeros(n + 1, dtype=np.int32)
    p = np.zeros(1, dtype=np.int32)
    st = lib().orc_graph_compress(n, _p(rp), _p(ci), float(mu), _p(perm), _p(bptr), _p(p))
    if st != OK:
        raise ValueError(f"orc_graph_compress failed ({st})")
    return perm[:n].copy(), bptr[: p[0] + 1].copy()


class BlockMatrix:
    """Exported block sparse row matrix (row-major dense blocks)."""

    def __init__(self, rb, cb, rowptr, colidx, vals, piv=None):
        self.rb, self.cb, self.rowptr, self.colidx, self.vals, self.piv = rb, cb, rowptr, colidx, vals, piv
        self.p, self.q = len(rb) - 1, len(cb) - 1
        rows = np.repeat(np.arange(self.p), np.diff(rowptr))
        sizes = (np.diff(rb)[rows].astype(np.int64) * np.diff(cb)[np.asarray(colidx, dtype=np.int64)])
        self.voff = np.zeros(len(colidx) + 1, dtype=np.int64)
        if sizes.size:
            np.cumsum(sizes, out=self.voff[1:])

    @property
    def nb(self):
        return len(self.colidx)

    def block(self, k):
        i = int(np.searchsorted(self.rowptr, k, side="right") - 1)
        m = self.rb[i + 1] - self.rb[i]
        j = self.colidx[k]
        n = self.cb[j + 1] - self.cb[j]
        return self.vals[self.voff[k]: self.voff[k + 1]].reshape(m, n)

    def dense(self):
        a = np.zeros((self.rb[-1], self.cb[-1]))
        for i in range(self.p):
            for k in range(self.rowptr[i], self.rowptr[i + 1]):
                j = self.colidx[k]
                a[self.rb[i]:self.rb[i + 1], self.cb[j]:self.cb[j + 1]] = self.block(k)
        return a


class Oracle:
    """Sequential FP64 VBARMS: compression result in, factors and solves out."""

    def __init__(self, n, rowptr, col, val, perm, bptr, levels, droptol, drop_schur=1, is_order=0, group_rows=0):
        rp, ci, v = _csr(rowptr, col, val)
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        bptr = np.ascontiguousarray(bptr, dtype=np.int32)
        dt = np.asarray(droptol, dtype=np.float64).ravel()
        if dt.size == 1:
            dt = np.full(levels + 1, dt[0])
        if dt.size < levels + 1:
            raise ValueError("droptol needs levels + 1 entries")
        self.n = n
        self._keep = (rp, ci, v, perm, bptr, dt)
        self.h = lib().orc_build(n, _p(rp), _p(ci), _p(v), _p(perm), _p(bptr), len(bptr) - 1,
                                 levels, _p(dt), drop_schur, is_order, group_rows)
        el = np.zeros(1, np.int32)
        eb = np.zeros(1, np.int32)
        self.status = lib().orc_status(self.h, _p(el), _p(eb))
        self.err_level, self.err_block = int(el[0]), int(eb[0])

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    @property
    def nlevels(self):
        return lib().orc_nlevels(self.h)

    def level_info(self, l):
        """p, n, nis (groups = pivot blocks of D), n_is, nis_sn (supernodes in the groups)."""
        info = np.zeros(5, np.int32)
        lib().orc_level_info(self.h, l, _p(info))
        return dict(p=int(info[0]), n=int(info[1]), nis=int(info[2]), n_is=int(info[3]), nis_sn=int(info[4]))

    def level_is(self, l):
        """The supernodes of the independent set, group after group."""
        k = self.level_info(l)["nis_sn"]
        out = np.zeros(max(k, 1), np.int32)
        lib().orc_level_is(self.h, l, _p(out))
        return out[:k]

    def level_groups(self, l):
        """Group pointers into level_is(l): group g is level_is(l)[gptr[g]:gptr[g+1]]."""
        k = self.level_info(l)["nis"]
        out = np.zeros(k + 1, np.int32)
        lib().orc_level_groups(self.h, l, _p(out))
        return out

    def level_scaling(self, l):
        n = self.level_info(l)["n"]
        s1 = np.zeros(max(n, 1))
        s2 = np.zeros(max(n, 1))
        lib().orc_level_scaling(self.h, l, _p(s1), _p(s2))
        return s1[:n], s2[:n]

    def matrix(self, which, level=0):
        dims = np.zeros(4, np.int64)
        st = lib().orc_matrix_dims(self.h, which, level, _p(dims))
        if st != OK:
            raise ValueError(f"no matrix {which} at level {level}")
        p, q, nb, nv = (int(x) for x in dims)
        rb = np.zeros(p + 1, np.int32)
        cb = np.zeros(q + 1, np.int32)
        rowptr = np.zeros(p + 1, np.int64)
        colidx = np.zeros(max(nb, 1), np.int32)
        vals = np.zeros(max(nv, 1))
        piv = None
        if which in (D, DL):
            piv = np.zeros(max(rb.size, 1) * 64, np.int32)
        lib().orc_matrix_get(self.h, which, level, _p(rb), _p(cb), _p(rowptr), _p(colidx), _p(vals),
                             None if piv is None else _p(piv))
        if piv is not None:
            piv = piv[: rb[-1]]
        return BlockMatrix(rb, cb, rowptr, colidx[:nb], vals[:nv], piv)

    def factor_nnz(self):
        return int(lib().orc_factor_nnz(self.h))

    def apply(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        st = lib().orc_apply(self.h, _p(x), _p(y))
        if st != OK:
            raise RuntimeError(f"orc_apply failed ({st})")
        return y


def fgmres(n, rowptr, col, val, b, precond: Oracle | None, tol=1e-8, restart=30, maxit=1000, x0=None):
    """Right-preconditioned FGMRES(m) with modified Gram-Schmidt.

    Returns (x, status, iterations, true relative residual, estimate history)."""
    rp, ci, v = _csr(rowptr, col, val)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    its = np.zeros(1, np.int32)
    rel = np.zeros(1)
    hist = np.zeros(maxit + 1)
    st = lib().orc_fgmres(None if precond is None else precond.h, n, _p(rp), _p(ci), _p(v), _p(b), _p(x),
                          float(tol), int(restart), int(maxit), _p(its), _p(rel), _p(hist))
    return x, st, int(its[0]), float(rel[0]), hist[: its[0] + 1]
