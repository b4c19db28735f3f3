"""Python binding of libvbarms.so (argument marshalling only).

Every step of the method runs in the HIP library; this module converts torch device
tensors into pointers, passes the current HIP stream and turns error codes into
exceptions.  It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VBARMS_LIB") or os.path.join(HERE, "libvbarms.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_HIP, ERR_OOM, ERR_SINGULAR, ERR_NAN, ERR_STATE = -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
IS_NATURAL, IS_WEIGHTED = 0, 1
MAX_LEVELS = 16
MAX_BLOCK = 32
NOALLOC_MAX_N = 1 << 21
# exportable matrices
M_A, M_AS, M_G, M_W, M_D, M_LAST, M_L, M_U, M_DL = range(9)
# timed kernel classes
K_SPMV, K_APPLY, K_ILUT, K_TRSV, K_ORTHO = range(5)
K_COUNT = 5
K_NAMES = ("spmv", "apply", "ilut_wave", "trsv_sweeps", "cgs_pass")
NFEAT = 8

_ERRNAMES = {ERR_ARG: "ERR_ARG", ERR_HIP: "ERR_HIP", ERR_OOM: "ERR_OOM", ERR_SINGULAR: "ERR_SINGULAR",
             ERR_NAN: "ERR_NAN", ERR_STATE: "ERR_STATE"}


class VbarmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


class CStats(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("max_block", C.c_int32), ("nnz_blocks", C.c_int64),
                ("av_bd", C.c_double), ("av_bs", C.c_double)]


class _FParams(C.Structure):
    _fields_ = [("levels", C.c_int32), ("droptol", C.c_double * (MAX_LEVELS + 1)), ("drop_schur", C.c_int32),
                ("is_order", C.c_int32), ("precision", C.c_int32), ("group_rows", C.c_int32)]


class SInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("true_relres", C.c_double), ("status", C.c_int32),
                ("fp64_refactor", C.c_int32)]


class FStats(C.Structure):
    _fields_ = [("compress_ms", C.c_double), ("factor_ms", C.c_double), ("solve_ms", C.c_double),
                ("factor_level_ms", C.c_double * MAX_LEVELS), ("ilut_ms", C.c_double), ("levels", C.c_int32),
                ("last_p", C.c_int32), ("factor_values", C.c_int64), ("nnz", C.c_int64),
                ("spmv_lanes", C.c_int32), ("ilut_waves", C.c_int32), ("ilut_attempts", C.c_int32),
                ("ilut_result_bytes", C.c_double), ("illcond_blocks", C.c_int32), ("fp64_fallback", C.c_int32)]


class KStat(C.Structure):
    _fields_ = [("calls", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double)]


# name -> (restype, argtypes)
_P = C.c_void_p
SIGNATURES = {
    "vbarms_create": (C.c_int, [C.POINTER(C.c_void_p), _P]),
    "vbarms_destroy": (C.c_int, [_P]),
    "vbarms_last_error": (C.c_char_p, [_P]),
    "vbarms_compress": (C.c_int, [_P, C.POINTER(_Csr), C.c_double, _P, _P, C.POINTER(CStats)]),
    "vbarms_set_partition": (C.c_int, [_P, C.POINTER(_Csr), _P, _P, C.c_int32, C.POINTER(CStats)]),
    "vbarms_compress_graph": (C.c_int, [_P, C.POINTER(_Csr), C.c_double, _P, _P, C.POINTER(CStats)]),
    "vbarms_factor": (C.c_int, [_P, C.POINTER(_FParams)]),
    "vbarms_error_location": (C.c_int, [_P, _P, _P]),
    "vbarms_apply": (C.c_int, [_P, _P, _P]),
    "vbarms_spmv": (C.c_int, [_P, _P, _P]),
    "vbarms_spmv_noalloc": (C.c_int, [_P, _P, _P]),
    "vbarms_solve": (C.c_int, [_P, _P, _P, C.c_double, C.c_int32, C.c_int32, C.POINTER(SInfo)]),
    "vbarms_get_stats": (C.c_int, [_P, C.POINTER(FStats)]),
    "vbarms_batch_create": (C.c_int, [C.POINTER(C.c_void_p), _P]),
    "vbarms_batch_destroy": (C.c_int, [_P]),
    "vbarms_batch_last_error": (C.c_char_p, [_P]),
    "vbarms_batch_handle": (C.c_void_p, [_P]),
    "vbarms_batch_factor": (C.c_int, [_P, C.c_int32, _P, C.c_double, C.POINTER(_FParams)]),
    "vbarms_batch_offsets": (C.c_int, [_P, _P]),
    "vbarms_batch_solve": (C.c_int, [_P, _P, _P, C.c_int32, C.c_double, C.c_int32, C.c_int32, _P]),
    "vbarms_set_fp64_fallback": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_double]),
    "vbarms_device_memory": (C.c_int, [_P]),
    "vbarms_set_graphs": (C.c_int, [_P, C.c_int32]),
    "vbarms_features": (C.c_int, [_P, C.POINTER(_Csr), _P]),
    "vbarms_mlp_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P]),
    "vbarms_mlp_destroy": (C.c_int, [_P]),
    "vbarms_mlp_last_error": (C.c_char_p, [_P]),
    "vbarms_mlp_num_params": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "vbarms_mlp_set_params": (C.c_int, [_P, _P]),
    "vbarms_mlp_get_params": (C.c_int, [_P, _P]),
    "vbarms_mlp_forward": (C.c_int, [_P, _P, C.c_int32, _P]),
    "vbarms_mlp_loss_grad": (C.c_int, [_P, _P, _P, C.c_int32, C.POINTER(C.c_float), _P]),
    "vbarms_mlp_adam_step": (C.c_int, [_P, C.c_float]),
    "vbarms_set_timing": (C.c_int, [_P, C.c_int32]),
    "vbarms_kernel_stats": (C.c_int, [_P, C.POINTER(KStat)]),
    "vbarms_num_levels": (C.c_int, [_P, _P]),
    "vbarms_level_info": (C.c_int, [_P, C.c_int32, _P]),
    "vbarms_level_is": (C.c_int, [_P, C.c_int32, _P]),
    "vbarms_level_groups": (C.c_int, [_P, C.c_int32, _P]),
    "vbarms_set_spmv_lanes": (C.c_int, [_P, C.c_int32]),
    "vbarms_level_scaling": (C.c_int, [_P, C.c_int32, _P, _P]),
    "vbarms_matrix_dims": (C.c_int, [_P, C.c_int32, C.c_int32, _P]),
    "vbarms_matrix_get": (C.c_int, [_P, C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P]),
}

_lib = None


def lib():
    """Loads libvbarms.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1508_02219_amd.build`")
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dev_ptr(t, dtype):
    import torch
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} tensor")
    return C.c_void_p(t.data_ptr())


@dataclass
class Exported:
    """A factor matrix in block-sparse-row form (host arrays, dense row-major blocks)."""
    rb: np.ndarray
    cb: np.ndarray
    rowptr: np.ndarray
    colidx: np.ndarray
    vals: np.ndarray
    piv: np.ndarray | None

    @property
    def p(self):
        return len(self.rb) - 1

    def block(self, k):
        """Dense block k (row-major) of the exported matrix."""
        if not hasattr(self, "_voff"):
            rows = np.repeat(np.arange(self.p), np.diff(self.rowptr))
            sizes = np.diff(self.rb)[rows].astype(np.int64) * np.diff(self.cb)[np.asarray(self.colidx, np.int64)]
            self._voff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        i = int(np.searchsorted(self.rowptr, k, side="right") - 1)
        j = int(self.colidx[k])
        m, n = self.rb[i + 1] - self.rb[i], self.cb[j + 1] - self.cb[j]
        return self.vals[self._voff[k]:self._voff[k + 1]].reshape(m, n)


class Solver:
    """One VBARMS handle bound to the current device and the current torch stream."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("VBARMS needs a ROCm GPU")
        self._torch = torch
        s = stream if stream is not None else torch.cuda.current_stream()
        self._stream = s
        h = C.c_void_p()
        rc = lib().vbarms_create(C.byref(h), C.c_void_p(s.cuda_stream))
        if rc != OK:
            raise VbarmsError(rc, "vbarms_create failed")
        self.h = h
        self.n = 0
        self._A = None

    def close(self):
        if getattr(self, "h", None) and not getattr(self, "_borrowed", False):
            lib().vbarms_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_not_converged=False):
        if rc == OK or (allow_not_converged and rc == NOT_CONVERGED):
            return rc
        msg = lib().vbarms_last_error(self.h)
        raise VbarmsError(rc, msg.decode() if msg else "")

    def _csr(self, rowptr, col, val):
        torch = self._torch
        n = rowptr.numel() - 1
        self._A = (rowptr, col, val)  # keep alive for the call
        return _Csr(n, int(col.numel()), _dev_ptr(rowptr, torch.int64), _dev_ptr(col, torch.int32),
                    _dev_ptr(val, torch.float64))

    # -- Step 1 -----------------------------------------------------------------------
    def compress(self, rowptr, col, val, tau):
        """Angle-based compression (Sec. 2.1). Device CSR in; returns (perm, bptr, stats)."""
        torch = self._torch
        A = self._csr(rowptr, col, val)
        n = A.n
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=rowptr.device)
        bptr = torch.empty(n + 1, dtype=torch.int32, device=rowptr.device)
        st = CStats()
        self._check(lib().vbarms_compress(self.h, C.byref(A), float(tau), _dev_ptr(perm, torch.int32),
                                          _dev_ptr(bptr, torch.int32), C.byref(st)))
        self.n = n
        return perm[:n], bptr[: st.nblocks + 1], st

    def compress_graph(self, rowptr, col, val, mu):
        """Graph-based compression with target block density mu (Sec. 2.2, Alg. 1)."""
        torch = self._torch
        A = self._csr(rowptr, col, val)
        n = A.n
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=rowptr.device)
        bptr = torch.empty(n + 1, dtype=torch.int32, device=rowptr.device)
        st = CStats()
        self._check(lib().vbarms_compress_graph(self.h, C.byref(A), float(mu), _dev_ptr(perm, torch.int32),
                                                _dev_ptr(bptr, torch.int32), C.byref(st)))
        self.n = n
        return perm[:n], bptr[: st.nblocks + 1], st

    def set_partition(self, rowptr, col, val, perm, bptr):
        torch = self._torch
        A = self._csr(rowptr, col, val)
        st = CStats()
        self._check(lib().vbarms_set_partition(self.h, C.byref(A), _dev_ptr(perm, torch.int32),
                                               _dev_ptr(bptr, torch.int32), bptr.numel() - 1, C.byref(st)))
        self.n = A.n
        return st

    # -- Steps 2-4 and the last level ---------------------------------------------------
    def factor(self, levels, droptol, drop_schur=1, precision=F64, is_order=IS_NATURAL, group_rows=0):
        p = _fparams(levels, droptol, drop_schur, precision, is_order, group_rows)
        self._check(lib().vbarms_factor(self.h, C.byref(p)))

    def error_location(self):
        lv, bk = C.c_int32(), C.c_int32()
        lib().vbarms_error_location(self.h, C.byref(lv), C.byref(bk))
        return lv.value, bk.value

    # -- application ----------------------------------------------------------------------
    def apply(self, x, out=None):
        torch = self._torch
        y = torch.empty_like(x) if out is None else out
        self._check(lib().vbarms_apply(self.h, _dev_ptr(x, torch.float64), _dev_ptr(y, torch.float64)))
        return y

    def set_spmv_lanes(self, lanes):
        """Lanes per scalar row of the product kernel (4, 8, 16 or 32), overriding the pick of
        the autotuner."""
        self._check(lib().vbarms_set_spmv_lanes(self.h, int(lanes)))

    def spmv(self, x, out=None):
        torch = self._torch
        y = torch.empty_like(x) if out is None else out
        self._check(lib().vbarms_spmv(self.h, _dev_ptr(x, torch.float64), _dev_ptr(y, torch.float64)))
        return y

    def spmv_noalloc(self, x, out):
        """y = A x through the allocation-free entry point (out must be preallocated)."""
        torch = self._torch
        self._check(lib().vbarms_spmv_noalloc(self.h, _dev_ptr(x, torch.float64), _dev_ptr(out, torch.float64)))
        return out

    def solve(self, b, x0=None, tol=1e-8, restart=30, maxit=1000):
        torch = self._torch
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        info = SInfo()
        rc = lib().vbarms_solve(self.h, _dev_ptr(b, torch.float64), _dev_ptr(x, torch.float64), float(tol),
                                int(restart), int(maxit), C.byref(info))
        self._check(rc, allow_not_converged=True)
        return x, info

    def set_fp64_fallback(self, enable=True, f32_iter_limit=100, min_pivot_ratio=1e-4):
        """FP32 safeguards: FP64 refactorization on ill-conditioned pivot blocks or stagnation."""
        self._check(lib().vbarms_set_fp64_fallback(self.h, 1 if enable else 0, int(f32_iter_limit),
                                                   float(min_pivot_ratio)))

    def stats(self):
        st = FStats()
        self._check(lib().vbarms_get_stats(self.h, C.byref(st)))
        return st

    def features(self, rowptr, col, val):
        """VBARMS_NFEAT features of a device CSR matrix (numpy float32)."""
        A = self._csr(rowptr, col, val)
        f = np.zeros(NFEAT, np.float32)
        self._check(lib().vbarms_features(self.h, C.byref(A), _np_ptr(f)))
        return f

    def set_graphs(self, enable=True):
        """Replay the last-level sweeps from a captured graph (default) or launch them eagerly."""
        self._check(lib().vbarms_set_graphs(self.h, 1 if enable else 0))

    def set_timing(self, enable=True):
        """Starts (and clears) or stops event timing of the kernel classes K_*."""
        self._check(lib().vbarms_set_timing(self.h, 1 if enable else 0))

    def kernel_stats(self):
        """{name: (calls, total ms, total algorithmic bytes)} since timing was enabled."""
        out = (KStat * K_COUNT)()
        self._check(lib().vbarms_kernel_stats(self.h, out))
        return {K_NAMES[c]: (int(out[c].calls), float(out[c].ms), float(out[c].bytes)) for c in range(K_COUNT)}

    # -- inspection -----------------------------------------------------------------------
    def num_levels(self):
        v = C.c_int32()
        self._check(lib().vbarms_num_levels(self.h, C.byref(v)))
        return v.value

    def level_info(self, level):
        info = np.zeros(5, np.int32)
        self._check(lib().vbarms_level_info(self.h, level, _np_ptr(info)))
        return dict(p=int(info[0]), n=int(info[1]), nis=int(info[2]), n_is=int(info[3]), nis_sn=int(info[4]))

    def level_is(self, level):
        k = self.level_info(level)["nis_sn"]
        out = np.zeros(max(k, 1), np.int32)
        self._check(lib().vbarms_level_is(self.h, level, _np_ptr(out)))
        return out[:k]

    def level_groups(self, level):
        k = self.level_info(level)["nis"]
        out = np.zeros(k + 1, np.int32)
        self._check(lib().vbarms_level_groups(self.h, level, _np_ptr(out)))
        return out

    def level_scaling(self, level):
        n = self.level_info(level)["n"]
        s1, s2 = np.zeros(max(n, 1)), np.zeros(max(n, 1))
        self._check(lib().vbarms_level_scaling(self.h, level, _np_ptr(s1), _np_ptr(s2)))
        return s1[:n], s2[:n]

    def matrix(self, which, level=0):
        dims = np.zeros(4, np.int64)
        self._check(lib().vbarms_matrix_dims(self.h, which, level, _np_ptr(dims)))
        p, q, nb, nv = (int(x) for x in dims)
        rb, cb = np.zeros(p + 1, np.int32), np.zeros(q + 1, np.int32)
        rowptr = np.zeros(p + 1, np.int64)
        colidx = np.zeros(max(nb, 1), np.int32)
        vals = np.zeros(max(nv, 1))
        # the pivot array has one entry per scalar row, never more than the m*m values
        piv = np.zeros(max(nv, 1), np.int32) if which in (M_D, M_DL) else None
        self._check(lib().vbarms_matrix_get(self.h, which, level, _np_ptr(rb), _np_ptr(cb), _np_ptr(rowptr),
                                            _np_ptr(colidx), _np_ptr(vals), None if piv is None else _np_ptr(piv)))
        if piv is not None:
            piv = piv[: rb[-1]]
        return Exported(rb, cb, rowptr, colidx[:nb], vals[:nv], piv)


def _fparams(levels, droptol, drop_schur=1, precision=F64, is_order=IS_NATURAL, group_rows=0):
    p = _FParams()
    p.levels = levels
    dt = np.asarray(droptol, dtype=np.float64).ravel()
    if dt.size == 1:
        dt = np.full(levels + 1, dt[0])
    for i in range(levels + 1):
        p.droptol[i] = float(dt[i])
    p.drop_schur = drop_schur
    p.is_order = is_order
    p.precision = precision
    p.group_rows = group_rows
    return p


class BatchSolver:
    """Several independent systems factored and solved through shared launches."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("VBARMS needs a ROCm GPU")
        self._torch = torch
        s = stream if stream is not None else torch.cuda.current_stream()
        b = C.c_void_p()
        rc = lib().vbarms_batch_create(C.byref(b), C.c_void_p(s.cuda_stream))
        if rc != OK:
            raise VbarmsError(rc, "vbarms_batch_create failed")
        self.b = b
        self.off = None

    def close(self):
        if getattr(self, "b", None):
            lib().vbarms_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_not_converged=False):
        if rc == OK or (allow_not_converged and rc == NOT_CONVERGED):
            return rc
        msg = lib().vbarms_batch_last_error(self.b)
        raise VbarmsError(rc, msg.decode() if msg else "")

    def factor(self, systems, tau, levels, droptol, drop_schur=1, precision=F64, is_order=IS_NATURAL, group_rows=0):
        """systems: list of (rowptr, col, val) device tensors."""
        torch = self._torch
        descs = (_Csr * len(systems))()
        self._keep = systems
        for q, (rp, ci, va) in enumerate(systems):
            descs[q] = _Csr(rp.numel() - 1, int(ci.numel()), _dev_ptr(rp, torch.int64), _dev_ptr(ci, torch.int32),
                            _dev_ptr(va, torch.float64))
        p = _fparams(levels, droptol, drop_schur, precision, is_order, group_rows)
        self._check(lib().vbarms_batch_factor(self.b, len(systems), descs, float(tau), C.byref(p)))
        off = np.zeros(len(systems) + 1, np.int64)
        self._check(lib().vbarms_batch_offsets(self.b, _np_ptr(off)))
        self.off = off
        return off

    def solve(self, B, X0=None, tol=1e-8, restart=30, maxit=1000):
        """B: device tensor [nrhs, N] (row r = right-hand side r of every system); returns
        (X, info) with info[r][s] the solver info of system s for right-hand side r."""
        torch = self._torch
        B = B.contiguous()
        nrhs = B.shape[0]
        X = torch.zeros_like(B) if X0 is None else X0.clone().contiguous()
        ns = len(self.off) - 1 if self.off is not None else 0
        info = (SInfo * max(1, nrhs * ns))()
        rc = lib().vbarms_batch_solve(self.b, _dev_ptr(B, torch.float64), _dev_ptr(X, torch.float64), nrhs,
                                      float(tol), int(restart), int(maxit), info)
        self._check(rc, allow_not_converged=True)
        return X, [[info[r * ns + q] for q in range(ns)] for r in range(nrhs)]

    def handle(self):
        """A Solver view of the combined system (apply, spmv, stats, exports); not owned."""
        sv = Solver.__new__(Solver)
        sv._torch = self._torch
        sv.h = C.c_void_p(lib().vbarms_batch_handle(self.b))
        sv.n = int(self.off[-1])
        sv._A = None
        sv._borrowed = True
        return sv


class Mlp:
    """The parameter-prediction network (FP32, trained by the library's kernels)."""

    def __init__(self, in_dim, hidden, depth, out_dim, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the MLP needs a ROCm GPU")
        self._torch = torch
        s = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        rc = lib().vbarms_mlp_create(C.byref(h), in_dim, hidden, depth, out_dim, C.c_void_p(s.cuda_stream))
        if rc != OK:
            raise VbarmsError(rc, "vbarms_mlp_create failed")
        self.h = h
        self.dims = (in_dim, hidden, depth, out_dim)
        n = C.c_int64()
        lib().vbarms_mlp_num_params(self.h, C.byref(n))
        self.num_params = int(n.value)

    def close(self):
        if getattr(self, "h", None):
            lib().vbarms_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != OK:
            msg = lib().vbarms_mlp_last_error(self.h)
            raise VbarmsError(rc, msg.decode() if msg else "")

    def set_params(self, p):
        t = self._torch.as_tensor(p, dtype=self._torch.float32, device="cuda").contiguous()
        assert t.numel() == self.num_params
        self._check(lib().vbarms_mlp_set_params(self.h, _dev_ptr(t, self._torch.float32)))

    def get_params(self):
        t = self._torch.empty(self.num_params, dtype=self._torch.float32, device="cuda")
        self._check(lib().vbarms_mlp_get_params(self.h, _dev_ptr(t, self._torch.float32)))
        return t

    def forward(self, x):
        torch = self._torch
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        y = torch.empty((x.shape[0], self.dims[3]), dtype=torch.float32, device="cuda")
        self._check(lib().vbarms_mlp_forward(self.h, _dev_ptr(x, torch.float32), x.shape[0], _dev_ptr(y, torch.float32)))
        return y

    def loss_grad(self, x, t, want_grad=True):
        torch = self._torch
        x = torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous()
        t = torch.as_tensor(t, dtype=torch.float32, device="cuda").contiguous()
        g = torch.empty(self.num_params, dtype=torch.float32, device="cuda") if want_grad else None
        loss = C.c_float()
        self._check(lib().vbarms_mlp_loss_grad(self.h, _dev_ptr(x, torch.float32), _dev_ptr(t, torch.float32),
                                               x.shape[0], C.byref(loss),
                                               None if g is None else _dev_ptr(g, torch.float32)))
        return float(loss.value), g

    def adam_step(self, lr):
        self._check(lib().vbarms_mlp_adam_step(self.h, C.c_float(lr)))


def device_memory():
    """{live, cached, peak, runtime_allocs} of the library's device memory cache (bytes, count)."""
    out = np.zeros(4, np.int64)
    rc = lib().vbarms_device_memory(_np_ptr(out))
    if rc != OK:
        raise VbarmsError(rc, "vbarms_device_memory failed")
    return dict(live=int(out[0]), cached=int(out[1]), peak=int(out[2]), runtime_allocs=int(out[3]))


def csr_to_device(system, device="cuda"):
    """Moves a host CSR (anything with rowptr/col/val numpy arrays) to device tensors."""
    import torch
    rp = torch.as_tensor(np.ascontiguousarray(system.rowptr, dtype=np.int64), device=device)
    ci = torch.as_tensor(np.ascontiguousarray(system.col, dtype=np.int32), device=device)
    va = torch.as_tensor(np.ascontiguousarray(system.val, dtype=np.float64), device=device)
    return rp, ci, va
