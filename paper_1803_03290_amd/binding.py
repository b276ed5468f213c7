"""ctypes binding of ``libgpcg.so``: same names as the C ABI, marshalling only."""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpcg.so")

CONVERGED, MAX_ITER, BREAKDOWN, NONFINITE, CONVERGED_ISLANDED, ISLANDED_NO_GEN, BAD_OUTAGE = range(7)
KIND_BP, KIND_BPP = 0, 1

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)


class GpcgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"gpcg error {code}: {msg}")
        self.code = code


class _Csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("rowptr", _i32p), ("col", _i32p), ("val", _f64p)]


class _Options(C.Structure):
    _fields_ = [("kind", C.c_int32), ("block", C.c_int32), ("base_max_iter", C.c_int32), ("lookahead", C.c_int32),
                ("zero_start", C.c_int32), ("reorder", C.c_int32), ("perm", _i32p)]


class Info(C.Structure):
    _fields_ = [
        ("n_bus", C.c_int32), ("m", C.c_int32), ("n_r", C.c_int32),
        ("nnz_a", C.c_int32), ("nnz_l", C.c_int32), ("nnz_u", C.c_int32),
        ("bandwidth", C.c_int32), ("block", C.c_int32), ("rows_per_step", C.c_int32),
        ("ring_fwd", C.c_int32), ("ring_bwd", C.c_int32), ("steps_fwd", C.c_int32), ("steps_bwd", C.c_int32),
        ("n_bridges", C.c_int32), ("base_iters", C.c_int32), ("base_resid", C.c_double),
        ("sym_factors", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes) of every exported symbol of include/gpcg.h
_VP = C.c_void_p
SIGNATURES = {
    "gpcg_last_error": (C.c_char_p, []),
    "gpcg_assemble": (C.c_int, [C.c_int32, C.c_int32, _i32p, _i32p, _f64p, _f64p, _i32p, _i32p, _i32p, _f64p,
                                C.c_int32, _i32p]),
    "gpcg_rcm": (C.c_int, [C.c_int32, C.c_int32, _i32p, _i32p, _i32p]),
    "gpcg_bridge_flags": (C.c_int, [_VP, _u8p]),
    "gpcg_get_perm": (C.c_int, [_VP, _i32p]),
    "gpcg_ilu0": (C.c_int, [C.POINTER(_Csr), _i32p, _i32p, _f64p, _i32p, _i32p, _i32p, _f64p, _i32p]),
    "gpcg_topology": (C.c_int, [C.c_int32, C.c_int32, _i32p, _i32p, _u8p, _i32p, _i32p, _i32p, _i32p]),
    "gpcg_setup": (C.c_int, [C.POINTER(_VP), C.c_int32, C.c_int32, _i32p, _i32p, _f64p, C.POINTER(_Csr),
                             C.POINTER(_Csr), C.POINTER(_Csr), _f64p, _f64p, C.POINTER(_Options), _VP]),
    "gpcg_destroy": (None, [_VP]),
    "gpcg_get_info": (C.c_int, [_VP, C.POINTER(Info)]),
    "gpcg_get_base": (C.c_int, [_VP, _u8p, _f64p]),
    "gpcg_solve_contingencies": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_double, C.c_int32, _VP, _VP, _VP, _VP,
                                           _VP, _VP]),
    "gpcg_solve_plain": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_double, C.c_int32, _VP, _VP, _VP, _VP, _VP, _VP]),
    "gpcg_solve_contingencies_noalloc": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_double, C.c_int32, _VP, _VP, _VP,
                                                   _VP, _VP, _VP]),
    "gpcg_solve_rhs": (C.c_int, [_VP, C.c_int32, _VP, _VP, C.c_int32, C.c_double, C.c_int32, _VP, _VP, _VP, _VP,
                                 _VP]),
    "gpcg_overload_gradients": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, C.c_double, C.c_double, C.c_int32, _VP,
                                          _VP, _VP, _VP, _VP]),
    "gpcg_weighted_rows": (C.c_int, [_VP, C.c_int32, C.c_int32, _VP, C.c_int32, _VP, _VP]),
    "gpcg_screen_overloads": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP, _VP]),
    "gpcg_batch_create": (C.c_int, [C.POINTER(_VP), C.c_int32, _VP, C.c_int32, C.c_int32, _i32p, _VP, _VP,
                                    C.c_double, C.c_int32, _VP, _VP, _VP, _VP, _VP]),
    "gpcg_batch_run": (C.c_int, [_VP]),
    "gpcg_batch_destroy": (None, [_VP]),
    "gpcg_batch_tune": (C.c_int, [C.c_int32, _VP, _i32p, _VP, _VP, C.c_double, C.c_int32, C.c_int32, _i32p,
                                  _i32p, C.c_int32, _f64p]),
    "gpcg_fdpf": (C.c_int, [_VP, _VP, C.c_int32, _VP, _VP, _VP, _VP, _VP, C.c_int32, C.c_double, C.c_int32, _VP,
                            _VP, _VP, _VP]),
    "gpcg_spmm": (C.c_int, [_VP, C.c_int32, _VP, _VP, _VP, _VP]),
    "gpcg_get_order": (C.c_int, [_VP, C.c_int32, _i32p]),
    "gpcg_get_sweeps": (C.c_int, [_VP, _i32p, C.POINTER(C.c_int64)]),
    "gpcg_set_timing": (C.c_int, [_VP, C.c_int]),
    "gpcg_get_timing": (C.c_int, [_VP, _f64p]),
}

_lib = None


def lib():
    """Load libgpcg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1803_03290_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise GpcgError(rc, lib().gpcg_last_error().decode())


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_i32p)


def _fp(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_f64p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Csr:
    """Host CSR matrix (int32 indices, float64 values)."""

    def __init__(self, rowptr, col, val):
        self.rowptr, self.col, self.val = _i32(rowptr), _i32(col), _f64(val)
        self.n = len(self.rowptr) - 1

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def _c(self):
        return _Csr(self.n, self.nnz, _ip(self.rowptr), _ip(self.col), _fp(self.val))

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


def assemble(n_bus, br_from, br_to, x, shunt=None, perm=None) -> Csr:
    """gpcg_assemble: reduced B' (or B'' with shunts), slack row/column
    dropped, rows in bus order or in ``perm``'s order."""
    f, t, xx = _i32(br_from), _i32(br_to), _f64(x)
    m = len(f)
    cap = n_bus - 1 + 2 * m
    rowptr = np.zeros(n_bus, np.int32)
    col = np.zeros(max(cap, 1), np.int32)
    val = np.zeros(max(cap, 1), np.float64)
    nnz = C.c_int32(0)
    sh = None if shunt is None else _f64(shunt)
    pm = None if perm is None else _i32(perm)
    _check(lib().gpcg_assemble(n_bus, m, _ip(f), _ip(t), _fp(xx), _fp(sh), None if pm is None else _ip(pm),
                               _ip(rowptr), _ip(col), _fp(val), cap, C.byref(nnz)))
    return Csr(rowptr, col[: nnz.value].copy(), val[: nnz.value].copy())


def rcm(n_bus, br_from, br_to) -> np.ndarray:
    """gpcg_rcm: the library's reverse Cuthill-McKee row order (bus of each
    reduced row)."""
    f, t = _i32(br_from), _i32(br_to)
    perm = np.zeros(n_bus - 1, np.int32)
    _check(lib().gpcg_rcm(n_bus, len(f), _ip(f), _ip(t), _ip(perm)))
    return perm


def ilu0(A: Csr):
    """gpcg_ilu0: zero-fill incomplete LU; returns (L strictly lower, U upper)."""
    n, nnz = A.n, A.nnz
    lr, ur = np.zeros(n + 1, np.int32), np.zeros(n + 1, np.int32)
    lc, uc = np.zeros(max(nnz, 1), np.int32), np.zeros(max(nnz, 1), np.int32)
    lv, uv = np.zeros(max(nnz, 1)), np.zeros(max(nnz, 1))
    nl, nu = C.c_int32(0), C.c_int32(0)
    a = A._c()
    _check(lib().gpcg_ilu0(C.byref(a), _ip(lr), _ip(lc), _fp(lv), C.byref(nl), _ip(ur), _ip(uc), _fp(uv),
                           C.byref(nu)))
    return (Csr(lr, lc[: nl.value].copy(), lv[: nl.value].copy()), Csr(ur, uc[: nu.value].copy(), uv[: nu.value].copy()))


def jacobi_factors(A: Csr):
    """Factors of the Jacobi preconditioner M = diag(A) in the library's
    factor format: L with no entries, U the diagonal (argument marshalling:
    the diagonal is copied out of A's arrays)."""
    n = len(A.rowptr) - 1
    rows = np.repeat(np.arange(n, dtype=np.int32), np.diff(A.rowptr))
    diag = A.val[A.col == rows]
    if len(diag) != n:
        raise ValueError("A must hold every diagonal entry once")
    L = Csr(np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    U = Csr(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), diag)
    return L, U


def topology(n_bus, br_from, br_to):
    """gpcg_topology: bridge flags, DFS pre-order, subtree sizes, island intervals."""
    f, t = _i32(br_from), _i32(br_to)
    m = len(f)
    isb = np.zeros(m, np.uint8)
    pre, sub = np.zeros(n_bus, np.int32), np.zeros(n_bus, np.int32)
    lo, hi = np.zeros(m, np.int32), np.zeros(m, np.int32)
    _check(lib().gpcg_topology(n_bus, m, _ip(f), _ip(t), isb.ctypes.data_as(_u8p), _ip(pre), _ip(sub), _ip(lo),
                               _ip(hi)))
    return dict(is_bridge=isb.astype(bool), pre=pre, subtree=sub, island_lo=lo, island_hi=hi)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A device context (gpcg_setup / gpcg_destroy) for one grid and one
    matrix kind.  Buses keep the caller's numbering in every input and
    output.  The row order of the reduced system is ``perm``: "rcm" (the
    default) lets gpcg_setup order the rows by its reverse Cuthill-McKee
    pass and form the ILU(0) itself; an array gives the bus of each row
    (A, L, U, if given, are in that order); None keeps the bus order.
    ``A`` defaults to the library's own assembly; ``L``, ``U`` to the
    ILU(0) the library forms; ``precond="jacobi"`` passes L = 0 and
    U = diag(A) instead (the Jacobi preconditioner of the GPCG listing,
    Section III.B).  ``zero_start`` starts every scenario from x0 = 0 (the
    listing of Section III.A) instead of the base state."""

    def __init__(self, n_bus, br_from, br_to, x, base_rhs=None, *, shunt=None, kind=KIND_BP, block=64,
                 theta_base=None, A: Csr | None = None, L: Csr | None = None, U: Csr | None = None, lookahead=0,
                 stream=None, precond="ilu0", zero_start=False, perm="rcm"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("a HIP GPU is required")
        self._lib = lib()
        self.n_bus, self.m, self.kind = int(n_bus), len(br_from), kind
        self.br_from, self.br_to, self.x = _i32(br_from), _i32(br_to), _f64(x)
        if precond not in ("ilu0", "jacobi"):
            raise ValueError(f"unknown preconditioner {precond!r}")
        reorder = False
        if isinstance(perm, str):
            if perm != "rcm":
                raise ValueError(f"unknown row order {perm!r}")
            if L is not None or U is not None:
                raise ValueError("factors come with their row order: pass perm as an array or None")
            if precond == "jacobi":
                perm = rcm(n_bus, br_from, br_to)
            else:
                perm, reorder = None, True
        pm = None if perm is None else _i32(perm)
        self.A = A if A is not None else assemble(n_bus, br_from, br_to, x, shunt, None if reorder else pm)
        if precond == "jacobi" and (L is None or U is None):
            L, U = jacobi_factors(self.A)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opt = _Options(kind, block, 0, lookahead, 1 if zero_start else 0, 1 if reorder else 0,
                       None if pm is None else _ip(pm))
        a = self.A._c()
        l = None if L is None else C.byref(L._c())
        u = None if U is None else C.byref(U._c())
        h = C.c_void_p()
        rhs = None if base_rhs is None else _f64(base_rhs)
        tb = None if theta_base is None else _f64(theta_base)
        self._keep = (pm, L, U)
        _check(self._lib.gpcg_setup(C.byref(h), self.n_bus, self.m, _ip(self.br_from), _ip(self.br_to),
                                    _fp(self.x), C.byref(a), l, u, _fp(rhs), _fp(tb),
                                    C.byref(opt), C.c_void_p(self.stream.cuda_stream)))
        self._h = h
        self.perm = np.zeros(self.n_bus - 1, np.int32)
        _check(self._lib.gpcg_get_perm(self._h, _ip(self.perm)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gpcg_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        I = Info()
        _check(self._lib.gpcg_get_info(self._h, C.byref(I)))
        return I.as_dict()

    def bridge_flags(self) -> np.ndarray:
        """gpcg_bridge_flags: bool[m]."""
        isb = np.zeros(self.m, np.uint8)
        _check(self._lib.gpcg_bridge_flags(self._h, isb.ctypes.data_as(_u8p)))
        return isb.astype(bool)

    def base(self):
        """(is_bridge[m] bool, theta_base[n_bus]) as NumPy arrays."""
        isb = np.zeros(self.m, np.uint8)
        th = np.zeros(self.n_bus)
        _check(self._lib.gpcg_get_base(self._h, isb.ctypes.data_as(_u8p), _fp(th)))
        return isb.astype(bool), th

    def alloc_outputs(self, n_out, flows=True, island=True, resid=True, device=None):
        import torch

        dev = device or torch.device("cuda", torch.cuda.current_device())
        out = dict(
            x=torch.empty((n_out, self.n_bus), dtype=torch.float64, device=dev),
            iters=torch.empty(n_out, dtype=torch.int32, device=dev),
            status=torch.empty(n_out, dtype=torch.int32, device=dev),
        )
        out["flows"] = torch.empty((n_out, self.m), dtype=torch.float64, device=dev) if flows else None
        out["island"] = torch.empty((n_out, self.n_bus), dtype=torch.uint8, device=dev) if island else None
        out["resid"] = torch.empty(n_out, dtype=torch.float64, device=dev) if resid else None
        return out

    def solve(self, outages, rhs, tol=1e-12, max_iter=20000, *, plain=False, out=None, flows=None, island=True,
              resid=True, noalloc=False):
        """gpcg_solve_contingencies (gpcg_solve_plain with ``plain``,
        gpcg_solve_contingencies_noalloc with ``noalloc``): outages and rhs
        are device tensors (int32[n_out], float64[n_bus]).  Returns the dict
        of device output tensors x, flows, iters, status, island, resid."""
        if flows is None:
            flows = self.kind == KIND_BP
        n_out = int(outages.shape[0])
        if out is None:
            out = self.alloc_outputs(n_out, flows, island, resid, outages.device)
        fn = (self._lib.gpcg_solve_plain if plain else
              self._lib.gpcg_solve_contingencies_noalloc if noalloc else self._lib.gpcg_solve_contingencies)
        _check(fn(self._h, n_out, _ptr(outages), _ptr(rhs), float(tol), int(max_iter), _ptr(out["x"]),
                  _ptr(out["flows"]), _ptr(out["iters"]), _ptr(out["status"]), _ptr(out["island"]),
                  _ptr(out["resid"])))
        return out

    def solve_rhs(self, outages, rhs_cols, tol=1e-12, max_iter=20000, *, island=False, resid=True, x=None):
        """gpcg_solve_rhs: scenario j solves A_c x = rhs_cols[j] (device
        float64[n_out, ld], ld >= n_bus) from x = 0.  Returns the dict of
        device tensors x, iters, status, island, resid."""
        import torch

        n_out = int(outages.shape[0])
        if rhs_cols.dim() != 2 or rhs_cols.shape[0] != n_out or rhs_cols.stride(1) != 1:
            raise ValueError("rhs_cols must be a row-major [n_out, ld] tensor")
        dev = outages.device
        out = {
            "x": x if x is not None else torch.empty((n_out, self.n_bus), dtype=torch.float64, device=dev),
            "iters": torch.empty(n_out, dtype=torch.int32, device=dev),
            "status": torch.empty(n_out, dtype=torch.int32, device=dev),
            "island": torch.empty((n_out, self.n_bus), dtype=torch.uint8, device=dev) if island else None,
            "resid": torch.empty(n_out, dtype=torch.float64, device=dev) if resid else None,
        }
        _check(self._lib.gpcg_solve_rhs(self._h, n_out, _ptr(outages), _ptr(rhs_cols), int(rhs_cols.stride(0)),
                                        float(tol), int(max_iter), _ptr(out["x"]), _ptr(out["iters"]),
                                        _ptr(out["status"]), _ptr(out["island"]), _ptr(out["resid"])))
        return out

    def overload_gradients(self, outages, P, F, kappa=20.0, tol=1e-12, max_iter=20000, *, grads=True):
        """gpcg_overload_gradients: per-scenario overload loss and (with
        grads) its gradients dL/dP [n_out, n_bus] and dL/dx [n_out, m].
        Returns the dict of device tensors loss, grad_p, grad_x, iters,
        status (iters and status: forward then adjoint, 2 n_out)."""
        import torch

        n_out = int(outages.shape[0])
        dev = outages.device
        f64 = dict(dtype=torch.float64, device=dev)
        out = {
            "loss": torch.empty(n_out, **f64),
            "grad_p": torch.empty((n_out, self.n_bus), **f64) if grads else None,
            "grad_x": torch.empty((n_out, self.m), **f64) if grads else None,
            "iters": torch.zeros(2 * n_out, dtype=torch.int32, device=dev),
            "status": torch.zeros(2 * n_out, dtype=torch.int32, device=dev),
        }
        _check(self._lib.gpcg_overload_gradients(self._h, n_out, _ptr(outages), _ptr(P), _ptr(F), float(kappa),
                                                 float(tol), int(max_iter), _ptr(out["loss"]), _ptr(out["grad_p"]),
                                                 _ptr(out["grad_x"]), _ptr(out["iters"]), _ptr(out["status"])))
        return out

    def weighted_rows(self, a, w, out):
        """gpcg_weighted_rows: out = w @ a for a row-major [n_rows, n_cols]."""
        if a.dim() != 2 or a.stride(1) != 1:
            raise ValueError("a must be a row-major 2-D tensor")
        _check(self._lib.gpcg_weighted_rows(self._h, int(a.shape[0]), int(a.shape[1]), _ptr(a), int(a.stride(0)),
                                            _ptr(w), _ptr(out)))
        return out

    def fdpf(self, bpp, outages, P, Q, theta0, V0, n_outer=3, tol=1e-12, max_iter=20000):
        """gpcg_fdpf with this (B') context and the B'' context ``bpp``:
        n_outer fast-decoupled iterations of every outage from (theta0, V0).
        Returns the dict of device tensors theta, V [n_out, n_bus], iters,
        status."""
        import torch

        n_out = int(outages.shape[0])
        dev = outages.device
        out = {
            "theta": torch.empty((n_out, self.n_bus), dtype=torch.float64, device=dev),
            "V": torch.empty((n_out, self.n_bus), dtype=torch.float64, device=dev),
            "iters": torch.empty(n_out, dtype=torch.int32, device=dev),
            "status": torch.empty(n_out, dtype=torch.int32, device=dev),
        }
        _check(self._lib.gpcg_fdpf(self._h, bpp._h, n_out, _ptr(outages), _ptr(P), _ptr(Q), _ptr(theta0), _ptr(V0),
                                   int(n_outer), float(tol), int(max_iter), _ptr(out["theta"]), _ptr(out["V"]),
                                   _ptr(out["iters"]), _ptr(out["status"])))
        return out

    def screen_overloads(self, flows, F):
        """gpcg_screen_overloads: per scenario the overloaded-branch count, the
        worst loading |f| / F and its branch (device tensors)."""
        import torch

        n_out = int(flows.shape[0])
        dev = flows.device
        out = {
            "count": torch.empty(n_out, dtype=torch.int32, device=dev),
            "worst": torch.empty(n_out, dtype=torch.float64, device=dev),
            "worst_branch": torch.empty(n_out, dtype=torch.int32, device=dev),
        }
        _check(self._lib.gpcg_screen_overloads(self._h, n_out, _ptr(flows), _ptr(F), _ptr(out["count"]),
                                               _ptr(out["worst"]), _ptr(out["worst_branch"])))
        return out

    def order(self, n_out) -> np.ndarray:
        """gpcg_get_order: scenario handed out j-th by the last solve's queue."""
        o = np.zeros(n_out, np.int32)
        _check(self._lib.gpcg_get_order(self._h, int(n_out), _ip(o)))
        return o

    def sweeps(self):
        """gpcg_get_sweeps: (waves, PCG iterations summed over the waves) of
        the last solve's launch."""
        w, n = C.c_int32(0), C.c_int64(0)
        _check(self._lib.gpcg_get_sweeps(self._h, C.byref(w), C.byref(n)))
        return int(w.value), int(n.value)

    def set_timing(self, enable=True):
        """gpcg_set_timing: bracket every solve's PCG kernels with HIP events."""
        _check(self._lib.gpcg_set_timing(self._h, int(bool(enable))))

    def pcg_ms(self) -> float:
        """gpcg_get_timing: PCG kernel time of the last solve, in ms."""
        v = C.c_double(0)
        _check(self._lib.gpcg_get_timing(self._h, C.byref(v)))
        return v.value

    def spmm(self, outages, p, q, pq=None):
        """gpcg_spmm on tile-interleaved device blocks."""
        _check(self._lib.gpcg_spmm(self._h, int(outages.shape[0]), _ptr(outages), _ptr(p), _ptr(q), _ptr(pq)))


def _ptr_array(tensors):
    arr = (C.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


class Batch:
    """gpcg_batch_create / gpcg_batch_run / gpcg_batch_destroy: the scenario
    lists of several contexts (different grids, one device and stream)
    solved by one launch of the tile kernel, captured in a HIP graph.
    ``outages`` and ``rhs`` are lists of device tensors (int32[n_out_i],
    float64[n_bus_i]); the batch keeps them and re-reads their contents on
    every ``run()``.  ``out[i]`` holds grid i's device output tensors."""

    def __init__(self, contexts, outages, rhs, block, tol=1e-12, max_iter=20000, *, flows=True, resid=True,
                 lookahead=0):
        import torch

        if not (len(contexts) == len(outages) == len(rhs)):
            raise ValueError("one outage list and one right-hand side per context")
        self._lib = lib()
        self.contexts, self.outages, self.rhs = list(contexts), list(outages), list(rhs)
        self.out = []
        for ctx, o in zip(self.contexts, self.outages):
            n = int(o.shape[0])
            dev = o.device
            self.out.append({
                "x": torch.empty((n, ctx.n_bus), dtype=torch.float64, device=dev),
                "flows": (torch.empty((n, ctx.m), dtype=torch.float64, device=dev)
                          if flows and ctx.kind == KIND_BP else None),
                "iters": torch.empty(n, dtype=torch.int32, device=dev),
                "status": torch.empty(n, dtype=torch.int32, device=dev),
                "resid": torch.empty(n, dtype=torch.float64, device=dev) if resid else None,
            })
        k = len(self.contexts)
        ctxs = (C.c_void_p * k)(*[c._h.value for c in self.contexts])
        n_outs = np.array([int(o.shape[0]) for o in self.outages], np.int32)
        self._keep = (ctxs, n_outs)
        h = C.c_void_p()
        _check(self._lib.gpcg_batch_create(
            C.byref(h), k, ctxs, int(block), int(lookahead), _ip(n_outs), _ptr_array(self.outages),
            _ptr_array(self.rhs),
            float(tol), int(max_iter), _ptr_array([d["x"] for d in self.out]),
            _ptr_array([d["flows"] for d in self.out]), _ptr_array([d["iters"] for d in self.out]),
            _ptr_array([d["status"] for d in self.out]), _ptr_array([d["resid"] for d in self.out])))
        self._h = h
        self.block = int(block)

    def run(self):
        _check(self._lib.gpcg_batch_run(self._h))
        return self.out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.gpcg_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_tune(contexts, outages, rhs, candidates=(4, 8, 16), tol=1e-12, max_iter=20000, reps=1):
    """gpcg_batch_tune: milliseconds per batch solve for each candidate tile
    shape, a block or a (block, lookahead) pair."""
    k = len(contexts)
    ctxs = (C.c_void_p * k)(*[c._h.value for c in contexts])
    n_outs = np.array([int(o.shape[0]) for o in outages], np.int32)
    pairs = [(c, 0) if np.isscalar(c) else tuple(c) for c in candidates]
    cand = np.array([b for b, _ in pairs], np.int32)
    look = np.array([lk for _, lk in pairs], np.int32)
    ms = np.zeros(len(cand))
    _check(lib().gpcg_batch_tune(k, ctxs, _ip(n_outs), _ptr_array(outages), _ptr_array(rhs), float(tol),
                                 int(max_iter), len(cand), _ip(cand), _ip(look), int(reps), _fp(ms)))
    return dict(zip(list(candidates), (float(v) for v in ms)))

