"""FP64 CPU oracle for the Schwarz-preconditioned GMRES solve.

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product path never
imports this package.  It shares no code with the GPU implementation.

The arithmetic lives in ``oracle.c`` (plain single-threaded C99); this file
only builds it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ASM_ORACLE_LIB names another build of oracle.c (the sanitizer test runs
# the pins against one built with AddressSanitizer and UBSan)
_LIB = os.environ.get("ASM_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, INVALID, OOM, SINGULAR, NONFINITE = 0, 1, -1, -2, -3, -4
KIND_NONE, KIND_CLASSICAL, KIND_TWO_LEVEL = 0, 1, 2
ADDITIVE, RESTRICTED = 0, 1
LOCAL_ILU0, LOCAL_EXACT = 0, 1
FIELD_NEAR_FAR, FIELD_NEAR, FIELD_FAR = 0, 1, 2
COARSE_NONE, COARSE_ADDITIVE, COARSE_TWO_STAGE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                        _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Opts(C.Structure):
    _fields_ = [("kind", C.c_int), ("combine", C.c_int), ("sx", C.c_int),
                ("sy", C.c_int), ("overlap", C.c_int),
                ("near", C.c_int * 3), ("far", C.c_int * 3), ("local", C.c_int),
                ("field", C.c_int), ("coarse", C.c_int), ("cbox", C.c_int * 3)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int),
                ("rel_res_true", C.c_double), ("rel_res_est", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_last_error.restype = C.c_char_p
        L.or_spmv.argtypes = [C.c_int, P, P, P, P, P]
        L.or_precond_setup.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P,
                                       C.POINTER(_Opts), C.POINTER(C.c_void_p)]
        L.or_precond_setup.restype = C.c_int
        L.or_precond_free.argtypes = [P]
        L.or_precond_apply.argtypes = [P, P, P]
        L.or_precond_apply.restype = C.c_int
        L.or_precond_nsub.argtypes = [P]
        L.or_precond_nsub.restype = C.c_int
        L.or_sub_sizes.argtypes = [P, C.c_int, P, P, P, P]
        L.or_sub_export.argtypes = [P, C.c_int, P, P, P, P, P, P, P]
        L.or_sub_solve.argtypes = [P, C.c_int, P, P]
        L.or_gmres.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P, P,
                               C.c_int, C.c_double, C.c_int, C.c_int,
                               C.POINTER(_Info), P]
        L.or_gmres.restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def last_error() -> str:
    return lib().or_last_error().decode()


class OracleError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"oracle status {status}: {msg}")
        self.status = status


@dataclass
class Matrix:
    nx: int
    ny: int
    nz: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray

    @staticmethod
    def from_system(s) -> "Matrix":
        return Matrix(s.nx, s.ny, s.nz,
                      np.ascontiguousarray(s.row_ptr, dtype=np.int32),
                      np.ascontiguousarray(s.col_idx, dtype=np.int32),
                      np.ascontiguousarray(s.vals, dtype=np.float64).reshape(-1, 3, 3))

    @property
    def N(self):
        return self.nx * self.ny * self.nz


def _check_sizes(A: Matrix, *vecs) -> None:
    """Array lengths the C code cannot see: row_ptr of N+1, col_idx and
    vals of row_ptr[N] blocks, vectors of 3N (INVALID otherwise)."""
    N = A.N
    ok = (A.nx > 0 and A.ny > 0 and A.nz > 0 and A.row_ptr.ndim == 1 and A.row_ptr.size == N + 1)
    if ok:
        nnzb = int(A.row_ptr[N])
        ok = (0 <= nnzb and A.col_idx.size == nnzb and A.vals.size == 9 * nnzb)
    ok = ok and all(v is None or v.size == 3 * N for v in vecs)
    if not ok:
        raise OracleError(INVALID, "array sizes do not match the grid")


def spmv(A: Matrix, x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    _check_sizes(A, x)
    y = np.empty(3 * A.N)
    lib().or_spmv(A.N, _p(A.row_ptr), _p(A.col_idx), _p(A.vals), _p(x), _p(y))
    return y


@dataclass
class Sub:
    n: int
    nfine: int
    ncoarse: int
    label: np.ndarray
    cell: np.ndarray
    owned: np.ndarray
    rp: np.ndarray
    ci: np.ndarray
    a: np.ndarray  # [nnz,3,3]
    f: np.ndarray  # [nnz,3,3] (zeros in exact mode)


class Precond:
    """Oracle preconditioner B (see oracle.c for the definitions)."""

    def __init__(self, A: Matrix, kind=KIND_CLASSICAL, combine=RESTRICTED,
                 sx=1, sy=1, overlap=1, near=(2, 2, 2), far=(4, 4, 4),
                 local=LOCAL_ILU0, field=FIELD_NEAR_FAR, coarse=COARSE_NONE, cbox=(4, 4, 4)):
        self.A = A
        _check_sizes(A)
        o = _Opts(kind, combine, sx, sy, overlap, (C.c_int * 3)(*near),
                  (C.c_int * 3)(*far), local, field, coarse, (C.c_int * 3)(*cbox))
        h = C.c_void_p()
        st = lib().or_precond_setup(A.nx, A.ny, A.nz, _p(A.row_ptr), _p(A.col_idx),
                                    _p(A.vals), C.byref(o), C.byref(h))
        if st != OK:
            raise OracleError(st, last_error())
        self._h = h
        self.kind = kind

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_precond_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def nsub(self) -> int:
        return lib().or_precond_nsub(self._h)

    def apply(self, r: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64)
        _check_sizes(self.A, r)
        z = np.empty(3 * self.A.N)
        st = lib().or_precond_apply(self._h, _p(r), _p(z))
        if st != OK:
            raise OracleError(st, last_error())
        return z

    def sub(self, s: int) -> Sub:
        if not 0 <= s < self.nsub:
            raise OracleError(INVALID, "subdomain out of range")
        n, nf, nc, nnz = (C.c_int(), C.c_int(), C.c_int(), C.c_int())
        lib().or_sub_sizes(self._h, s, C.byref(n), C.byref(nf), C.byref(nc), C.byref(nnz))
        N = self.A.N
        label = np.empty(N, np.int32)
        cell = np.empty(max(nf.value, 1), np.int32)
        owned = np.empty(max(nf.value, 1), np.int32)
        rp = np.empty(n.value + 1, np.int32)
        ci = np.empty(max(nnz.value, 1), np.int32)
        a = np.empty((max(nnz.value, 1), 3, 3))
        f = np.zeros((max(nnz.value, 1), 3, 3))
        lib().or_sub_export(self._h, s, _p(label), _p(cell), _p(owned), _p(rp), _p(ci),
                            _p(a), _p(f))
        k = nnz.value
        return Sub(n.value, nf.value, nc.value, label, cell[:nf.value], owned[:nf.value],
                   rp, ci[:k], a[:k], f[:k])

    def sub_solve(self, s: int, rh: np.ndarray) -> np.ndarray:
        rh = np.ascontiguousarray(rh, dtype=np.float64)
        if not 0 <= s < self.nsub:
            raise OracleError(INVALID, "subdomain out of range")
        n, nf, nc, nnz = (C.c_int(), C.c_int(), C.c_int(), C.c_int())
        lib().or_sub_sizes(self._h, s, C.byref(n), C.byref(nf), C.byref(nc), C.byref(nnz))
        if rh.size != 3 * n.value:
            raise OracleError(INVALID, "right-hand side of another size")
        xh = np.empty_like(rh)
        lib().or_sub_solve(self._h, s, _p(rh), _p(xh))
        return xh


@dataclass
class Result:
    x: np.ndarray
    status: int
    iters: int
    cycles: int
    rel_res_true: float
    rel_res_est: float
    hist: np.ndarray


def gmres(A: Matrix, P: Precond, b: np.ndarray, x0: np.ndarray | None = None, *,
          restart=30, rtol=1e-6, max_iters=10000, fixed_iters=0) -> Result:
    """Restarted right-preconditioned GMRES (see or_gmres in oracle.c)."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(3 * A.N) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    _check_sizes(A, b, x)
    if P.A is not A and P.A.N != A.N:
        raise OracleError(INVALID, "preconditioner of another grid")
    info = _Info()
    hist = np.full(max(max_iters, fixed_iters) + 1, np.nan)
    st = lib().or_gmres(A.nx, A.ny, A.nz, _p(A.row_ptr), _p(A.col_idx), _p(A.vals),
                        P.handle, _p(b), _p(x), restart, rtol, max_iters, fixed_iters,
                        C.byref(info), _p(hist))
    if st < 0:
        raise OracleError(st, last_error())
    return Result(x, st, info.iters, info.cycles, info.rel_res_true, info.rel_res_est,
                  hist[:info.iters + 1])
