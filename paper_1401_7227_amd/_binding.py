"""ctypes binding of libasm_mi355x.so (argument marshalling only).

Every step of the solve runs in the library's HIP kernels; torch is used only
for device memory and the current HIP stream.  The library must be built
(``paper_1401_7227_amd.build.build()``); importing fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libasm_mi355x.so")

OK, NOT_CONVERGED = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20  # ASM_NOALLOC_SCRATCH_BYTES
ERR_INVALID, ERR_OOM, ERR_SINGULAR_PIVOT, ERR_NONFINITE, ERR_HIP = -1, -2, -3, -4, -5
KIND_NONE, KIND_CLASSICAL, KIND_TWO_LEVEL = 0, 1, 2
ADDITIVE, RESTRICTED = 0, 1
FP64, FP32 = 0, 1
FIELD_NEAR_FAR, FIELD_NEAR, FIELD_FAR = 0, 1, 2
COARSE_NONE, COARSE_ADDITIVE, COARSE_TWO_STAGE = 0, 1, 2
LOCAL_ILU0, LOCAL_EXACT = 0, 1

STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_INVALID", -2: "ERR_OOM",
                -3: "ERR_SINGULAR_PIVOT", -4: "ERR_NONFINITE", -5: "ERR_HIP"}

EXPORTED = ["asm_create_system", "asm_update_values", "asm_spmv", "asm_setup_precond",
            "asm_refactor", "asm_precond_apply", "asm_precond_get_stats",
            "asm_precond_export_sub", "asm_solve", "asm_solve_graph", "asm_solve_noalloc", "asm_solve_batch",
            "asm_destroy_precond",
            "asm_destroy_system", "asm_last_error", "asm_profile_enable", "asm_profile_read",
            "asm_precond_clone", "asm_server_create", "asm_server_submit", "asm_server_poll",
            "asm_server_get_state", "asm_server_destroy", "asm_tuning_get", "asm_tuning_set",
            "asm_batch_order_set", "asm_batch_tuning_last", "asm_set_allocator"]

SERVER_MAX_SOLVES = 8
SERVER_MAX_ACTIVE = 1024

PHASES = ["ilu_apply", "lump", "combine", "spmv", "dots", "update", "residual", "other"]


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


class PrecondOpts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("combine", C.c_int32), ("sx", C.c_int32),
                ("sy", C.c_int32), ("overlap", C.c_int32), ("near_box", C.c_int32 * 3),
                ("far_box", C.c_int32 * 3), ("precision", C.c_int32), ("field", C.c_int32),
                ("coarse", C.c_int32), ("coarse_box", C.c_int32 * 3), ("local", C.c_int32)]


class PrecondStats(C.Structure):
    _fields_ = [("nsub", C.c_int32), ("ext_rows", C.c_int64), ("coarse_rows", C.c_int64),
                ("factor_blocks", C.c_int64), ("fine_row_blocks", C.c_int64),
                ("max_levels", C.c_int32),
                ("device_bytes", C.c_int64), ("sweep_steps", C.c_int64), ("reloaded_rows", C.c_int64),
                ("split_rows", C.c_int64)]


class SolveOpts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("rtol", C.c_double), ("max_iters", C.c_int32),
                ("fixed_iters", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("cycles", C.c_int32), ("rel_res_true", C.c_double),
                ("rel_res_est", C.c_double)]


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * 8), ("ms", C.c_double * 8)]


TUNE_SOURCES = {0: "default", 1: "timed", 2: "cached", 3: "set"}


class Tuning(C.Structure):
    _fields_ = [("spmv_rows", C.c_int32), ("red_blocks", C.c_int32), ("source", C.c_int32),
                ("restart", C.c_int32), ("spmv_us", C.c_double * 3), ("krylov_us", C.c_double * 4)]


BATCH_ORDER_TUNE, BATCH_ORDER_SUBMITTED, BATCH_ORDER_LARGEST_FIRST = -1, 0, 1


class BatchTuning(C.Structure):
    _fields_ = [("order", C.c_int32), ("source", C.c_int32), ("ns_per_row_step", C.c_double * 2)]


class ServerOpts(C.Structure):
    _fields_ = [("solve", SolveOpts), ("hbm_budget_bytes", C.c_int64), ("max_active", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("tag", C.c_int64), ("grid", Grid), ("nb", C.c_int32), ("nnzb", C.c_int64),
                ("row_ptr_dev", C.c_void_p), ("col_idx_dev", C.c_void_p), ("precond", PrecondOpts),
                ("nsolves", C.c_int32), ("vals_dev", C.c_void_p * SERVER_MAX_SOLVES),
                ("b_dev", C.c_void_p * SERVER_MAX_SOLVES), ("x_dev", C.c_void_p * SERVER_MAX_SOLVES)]


class Completion(C.Structure):
    _fields_ = [("tag", C.c_int64), ("status", C.c_int32), ("solves", C.c_int32),
                ("iters", C.c_int32), ("plan_cached", C.c_int32), ("rel_res_true", C.c_double)]


class ServerState(C.Structure):
    _fields_ = [("queued", C.c_int32), ("running", C.c_int32), ("iterating", C.c_int32),
                ("completed_unread", C.c_int32), ("cached_plans", C.c_int32),
                ("bytes_in_use", C.c_int64), ("plan_builds", C.c_int64), ("plan_hits", C.c_int64)]


_lib = None
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p)
_alloc_hooks = None  # the registered callbacks (kept alive while set)


def load() -> C.CDLL:
    """Loads the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1401_7227_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    V = C.c_void_p
    L.asm_last_error.restype = C.c_char_p
    L.asm_create_system.argtypes = [C.POINTER(Grid), C.c_int32, C.c_int64, V, V, V, V,
                                    C.POINTER(V)]
    L.asm_update_values.argtypes = [V, V, V]
    L.asm_spmv.argtypes = [V, V, V, V]
    L.asm_setup_precond.argtypes = [V, C.POINTER(PrecondOpts), V, C.POINTER(V)]
    L.asm_refactor.argtypes = [V, V]
    L.asm_precond_apply.argtypes = [V, V, V, V]
    L.asm_precond_get_stats.argtypes = [V, C.POINTER(PrecondStats)]
    L.asm_precond_export_sub.argtypes = [V, C.c_int32, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), V, V, V, V, V]
    L.asm_solve.argtypes = [V, V, V, V, C.POINTER(SolveOpts), V, C.POINTER(SolveInfo)]
    L.asm_solve_graph.argtypes = [V, V, V, V, C.POINTER(SolveOpts), V, C.POINTER(SolveInfo)]
    L.asm_solve_batch.argtypes = [C.c_int32, C.POINTER(V), C.POINTER(V), C.POINTER(V), C.POINTER(V),
                                  C.POINTER(SolveOpts), V, C.POINTER(SolveInfo), C.POINTER(C.c_int32)]
    L.asm_profile_enable.argtypes = [V, C.c_int32]
    L.asm_profile_read.argtypes = [V, C.POINTER(Profile), C.c_int32]
    L.asm_precond_clone.argtypes = [V, V, V, C.POINTER(V)]
    L.asm_tuning_get.argtypes = [V, C.POINTER(Tuning)]
    L.asm_tuning_set.argtypes = [V, C.c_int32, C.c_int32]
    L.asm_batch_order_set.argtypes = [C.c_int32]
    L.asm_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, V]
    L.asm_batch_tuning_last.argtypes = [C.POINTER(BatchTuning)]
    L.asm_server_create.argtypes = [C.POINTER(ServerOpts), V, C.POINTER(V)]
    L.asm_server_submit.argtypes = [V, C.POINTER(Request)]
    L.asm_server_poll.argtypes = [V, C.c_int32, C.POINTER(Completion), C.POINTER(C.c_int32)]
    L.asm_server_get_state.argtypes = [V, C.POINTER(ServerState)]
    L.asm_server_destroy.argtypes = [V]
    L.asm_destroy_precond.argtypes = [V]
    L.asm_destroy_system.argtypes = [V]
    for name in EXPORTED:
        if name != "asm_last_error":
            getattr(L, name).restype = C.c_int
    L.asm_destroy_precond.restype = None
    L.asm_destroy_system.restype = None
    L.asm_server_destroy.restype = None
    _lib = L
    return L


class AsmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st: int) -> int:
    if st < 0:
        raise AsmError(st, load().asm_last_error().decode())
    return st


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype) -> torch.Tensor:
    if isinstance(t, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(t))
    t = t.to(device="cuda", dtype=dtype)
    return t.contiguous()


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _checked(t, dtype, n: int, name: str) -> torch.Tensor:
    """A tensor the library reads or writes through a bare pointer: the C
    side cannot see its size, so it must be a contiguous tensor of `dtype`
    on the current GPU with exactly n elements."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.device.type != "cuda" or t.device.index != torch.cuda.current_device():
        raise ValueError(f"{name}: must live on the current GPU (cuda:{torch.cuda.current_device()}), not {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} elements, expected {n}")
    return t


def _vec(t, n: int, name: str) -> torch.Tensor:
    """An input vector (array or tensor) as a contiguous float64 tensor on
    the GPU with n elements."""
    return _checked(_dev(t, torch.float64), torch.float64, n, name)


def _out(t, n: int, name: str) -> torch.Tensor:
    """An output vector: written in place, so never converted."""
    return _checked(t, torch.float64, n, name)


class System:
    """Device copy of A (= -J) in the library's own layout."""

    def __init__(self, nx, ny, nz, row_ptr, col_idx, vals):
        L = load()
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        rp = _dev(row_ptr, torch.int32)  # its length gives nb, which the library checks against the grid
        ci = _dev(col_idx, torch.int32)
        self.nnzb = int(ci.numel())
        v = _checked(_dev(vals, torch.float64).reshape(-1), torch.float64, 9 * self.nnzb, "vals")
        h = C.c_void_p()
        g = Grid(nx, ny, nz)
        _check(L.asm_create_system(C.byref(g), int(rp.numel()) - 1, self.nnzb, _ptr(rp),
                                   _ptr(ci), _ptr(v), _stream(), C.byref(h)))
        self._h = h

    @staticmethod
    def from_generated(s) -> "System":
        return System(s.nx, s.ny, s.nz, s.row_ptr, s.col_idx, s.vals)

    @property
    def handle(self):
        return self._h

    def update_values(self, vals):
        v = _checked(_dev(vals, torch.float64).reshape(-1), torch.float64, 9 * self.nnzb, "vals")
        _check(load().asm_update_values(self._h, _ptr(v), _stream()))

    def spmv(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        x = _vec(x, 3 * self.N, "x")
        y = torch.empty_like(x) if out is None else _out(out, 3 * self.N, "out")
        _check(load().asm_spmv(self._h, _ptr(x), _ptr(y), _stream()))
        return y

    def profile(self, enable: bool = True, phases=None):
        """Turns HIP-event timing of solve phases on (all, or the named
        phases) or off."""
        mask = 0
        if enable:
            mask = 0xFF if phases is None else sum(1 << PHASES.index(p) for p in phases)
        _check(load().asm_profile_enable(self._h, mask))

    def profile_read(self, reset: bool = True) -> dict:
        """{phase: (launches, device ms)} accumulated since the last reset."""
        p = Profile()
        _check(load().asm_profile_read(self._h, C.byref(p), 1 if reset else 0))
        return {name: (int(p.launches[k]), float(p.ms[k])) for k, name in enumerate(PHASES)}

    def tuning(self) -> dict:
        """The system's launch-shape choice: SpMV rows per thread, Krylov
        partial-sum blocks, where the choice came from, and the candidate
        timings (microseconds) it was made from."""
        t = Tuning()
        _check(load().asm_tuning_get(self._h, C.byref(t)))
        return {"spmv_rows": int(t.spmv_rows), "red_blocks": int(t.red_blocks),
                "source": TUNE_SOURCES.get(int(t.source), str(t.source)), "restart": int(t.restart),
                "spmv_us": {r: float(t.spmv_us[k]) for k, r in enumerate((1, 2, 4))},
                "krylov_us": {b: float(t.krylov_us[k]) for k, b in enumerate((512, 1024, 2048, 4096))}}

    def set_tuning(self, spmv_rows: int = 0, red_blocks: int = 0):
        """Fixes the launch-shape choice; (0, 0) makes the next solve time
        the candidates again."""
        _check(load().asm_tuning_set(self._h, int(spmv_rows), int(red_blocks)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().asm_destroy_system(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Export:
    n: int
    rp: np.ndarray
    ci: np.ndarray
    a: np.ndarray
    f: np.ndarray
    label: np.ndarray


class Precond:
    """Schwarz preconditioner B (classical or two-level) on a System."""

    def __init__(self, system: System, kind=KIND_CLASSICAL, combine=RESTRICTED, sx=1, sy=1,
                 overlap=1, near=(2, 2, 2), far=(4, 4, 4), precision=FP64, field=FIELD_NEAR_FAR,
                 coarse=COARSE_NONE, cbox=(4, 4, 4), local=LOCAL_ILU0, *, _clone_of=None):
        L = load()
        self.system = system
        h = C.c_void_p()
        if _clone_of is not None:
            _check(L.asm_precond_clone(_clone_of.handle, system.handle, _stream(), C.byref(h)))
            self._h = h
            self.kind = _clone_of.kind
            return
        o = PrecondOpts(kind, combine, sx, sy, overlap, (C.c_int32 * 3)(*near),
                        (C.c_int32 * 3)(*far), precision, field, coarse, (C.c_int32 * 3)(*cbox), local)
        _check(L.asm_setup_precond(system.handle, C.byref(o), _stream(), C.byref(h)))
        self._h = h
        self.kind = kind

    def clone(self, system: System) -> "Precond":
        """The preconditioner of `system` (same grid and pattern) on this
        one's plan: shared pattern-only state, own factors."""
        return Precond(system, _clone_of=self)

    @property
    def handle(self):
        return self._h

    def refactor(self):
        _check(load().asm_refactor(self._h, _stream()))

    def apply(self, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        n = 3 * self.system.N
        r = _vec(r, n, "r")
        z = torch.empty_like(r) if out is None else _out(out, n, "out")
        _check(load().asm_precond_apply(self._h, _ptr(r), _ptr(z), _stream()))
        return z

    def stats(self) -> dict:
        st = PrecondStats()
        _check(load().asm_precond_get_stats(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in PrecondStats._fields_}

    def export_sub(self, s: int) -> Export:
        L = load()
        n, nnz = C.c_int32(), C.c_int32()
        _check(L.asm_precond_export_sub(self._h, s, C.byref(n), C.byref(nnz), None, None, None,
                                        None, None))
        rp = np.empty(n.value + 1, np.int32)
        ci = np.empty(max(nnz.value, 1), np.int32)
        a = np.empty((max(nnz.value, 1), 3, 3))
        f = np.empty((max(nnz.value, 1), 3, 3))
        lab = np.empty(self.system.N, np.int32)
        p = lambda arr: arr.ctypes.data_as(C.c_void_p)  # noqa: E731
        _check(L.asm_precond_export_sub(self._h, s, C.byref(n), C.byref(nnz), p(rp), p(ci), p(a),
                                        p(f), p(lab)))
        k = nnz.value
        return Export(n.value, rp, ci[:k], a[:k], f[:k], lab)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().asm_destroy_precond(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Info:
    status: int
    iters: int
    cycles: int
    rel_res_true: float
    rel_res_est: float


def solve(system: System, precond: Precond, b, x0=None, *, restart=30, rtol=1e-6,
          max_iters=10000, fixed_iters=0, out: torch.Tensor | None = None, graph=False, noalloc=False):
    """Solves A x = b; returns (x, Info).  b, x0: device tensors or arrays.
    graph: every restart cycle runs as one captured HIP graph with the
    convergence test on the device (asm_solve_graph).  noalloc: the solve
    whose work arrays live in the library's fixed device array
    (asm_solve_noalloc; pass `out` to allocate nothing here either)."""
    if graph and noalloc:
        raise ValueError("graph and noalloc are separate entry points")
    n = 3 * system.N
    b = _vec(b, n, "b")
    if out is not None:
        x = _out(out, n, "out")
        if x0 is not None:
            x.copy_(_vec(x0, n, "x0"))
    else:
        x = torch.zeros_like(b) if x0 is None else _vec(x0, n, "x0").clone()
    o = SolveOpts(restart, rtol, max_iters, fixed_iters)
    info = SolveInfo()
    fn = load().asm_solve_graph if graph else (load().asm_solve_noalloc if noalloc else load().asm_solve)
    st = _check(fn(system.handle, precond.handle, _ptr(b), _ptr(x), C.byref(o), _stream(), C.byref(info)))
    return x, Info(st, info.iters, info.cycles, info.rel_res_true, info.rel_res_est)


def use_torch_allocator(enable: bool = True):
    """Routes the device arrays of handles created from now on through
    torch's caching allocator (enable=False: back to hipMalloc/hipFree).
    Handles keep the allocator they were created with."""
    global _alloc_hooks
    L = load()
    if not enable:
        _check(L.asm_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
        _alloc_hooks = None
        return

    def _alloc(nbytes, device, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device))
        except Exception:  # out of memory: the library reports ASM_ERR_OOM
            return None

    def _free(ptr, nbytes, device, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    hooks = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(L.asm_set_allocator(hooks[0], hooks[1], None))
    _alloc_hooks = hooks


def batch_order_set(order: int):
    """Order of the systems in batched launches: BATCH_ORDER_TUNE (default),
    BATCH_ORDER_SUBMITTED or BATCH_ORDER_LARGEST_FIRST (process-wide)."""
    _check(load().asm_batch_order_set(int(order)))


def batch_tuning_last() -> dict:
    """The order this thread's last solve_batch used, where the choice came
    from and the timings (ns per block row and step) of both orders."""
    t = BatchTuning()
    _check(load().asm_batch_tuning_last(C.byref(t)))
    return {"order": "largest_first" if t.order == BATCH_ORDER_LARGEST_FIRST else "submitted",
            "source": TUNE_SOURCES.get(int(t.source), str(t.source)),
            "ns_per_row_step": {"submitted": float(t.ns_per_row_step[0]),
                                "largest_first": float(t.ns_per_row_step[1])}}


def solve_batch(systems, preconds, bs, x0s=None, *, restart=30, rtol=1e-6, max_iters=10000, fixed_iters=0):
    """Solves independent systems together (one set of launches per step for
    all of them).  Returns ([x], [Info]); each equals solve() of that system."""
    n = len(systems)
    if n == 0:
        return [], []
    if len(preconds) != n or len(bs) != n or (x0s is not None and len(x0s) != n):
        raise ValueError("one preconditioner, b (and x0) per system")
    bs = [_vec(b, 3 * S.N, f"bs[{i}]") for i, (b, S) in enumerate(zip(bs, systems))]
    xs = []
    for i in range(n):
        if x0s is None or x0s[i] is None:
            xs.append(torch.zeros_like(bs[i]))
        else:
            xs.append(_vec(x0s[i], 3 * systems[i].N, f"x0s[{i}]").clone())
    V = C.c_void_p
    hs = (V * n)(*[s.handle.value for s in systems])
    ps = (V * n)(*[p.handle.value for p in preconds])
    bp = (V * n)(*[b.data_ptr() for b in bs])
    xp = (V * n)(*[x.data_ptr() for x in xs])
    o = SolveOpts(restart, rtol, max_iters, fixed_iters)
    infos = (SolveInfo * n)()
    stat = (C.c_int32 * n)()
    _check(load().asm_solve_batch(n, hs, ps, bp, xp, C.byref(o), _stream(), infos, stat))
    return xs, [Info(int(stat[i]), infos[i].iters, infos[i].cycles, infos[i].rel_res_true,
                     infos[i].rel_res_est) for i in range(n)]


def precond_opts(kind=KIND_TWO_LEVEL, combine=RESTRICTED, sx=1, sy=1, overlap=1, near=(2, 2, 2),
                 far=(4, 4, 4), precision=FP64, field=FIELD_NEAR_FAR, coarse=COARSE_NONE,
                 cbox=(4, 4, 4), local=LOCAL_ILU0) -> PrecondOpts:
    return PrecondOpts(kind, combine, sx, sy, overlap, (C.c_int32 * 3)(*near), (C.c_int32 * 3)(*far),
                       precision, field, coarse, (C.c_int32 * 3)(*cbox), local)


class Server:
    """Request server of the library (asm_server_*): requests queue, are
    admitted within a device-memory budget, and their solves iterate together.
    Tensors handed to submit() are kept alive here until their completion."""

    def __init__(self, *, restart=30, rtol=1e-6, max_iters=10000, budget_bytes=0, max_active=256):
        L = load()
        o = ServerOpts(SolveOpts(restart, rtol, max_iters, 0), budget_bytes, max_active)
        h = C.c_void_p()
        _check(L.asm_server_create(C.byref(o), _stream(), C.byref(h)))
        self._h = h
        self._live = {}

    def submit(self, tag: int, grid, row_ptr, col_idx, popts: PrecondOpts, vals, bs, xs):
        """grid (nx, ny, nz); row_ptr, col_idx: int32 device tensors; vals, bs,
        xs: lists of float64 device tensors, one per solve (xs hold x0 and
        receive the solutions)."""
        k = len(vals)
        if tag in self._live:
            # the library rejects it too; checked here first so the live
            # request's tensors are never released early
            raise ValueError(f"tag {tag} is in use by a live request")
        if not (1 <= k <= SERVER_MAX_SOLVES and len(bs) == k and len(xs) == k):
            raise ValueError("one values, b and x tensor per solve, 1..8 solves")
        nb = row_ptr.numel() - 1  # the library checks it against the grid
        _checked(row_ptr, torch.int32, nb + 1, "row_ptr")
        nnzb = col_idx.numel()
        _checked(col_idx, torch.int32, nnzb, "col_idx")
        for i in range(k):
            _checked(vals[i], torch.float64, 9 * nnzb, f"vals[{i}]")
            _checked(bs[i], torch.float64, 3 * nb, f"bs[{i}]")
            _checked(xs[i], torch.float64, 3 * nb, f"xs[{i}]")
        r = Request()
        r.tag = tag
        r.grid = Grid(*grid)
        r.nb = nb
        r.nnzb = nnzb
        r.row_ptr_dev = row_ptr.data_ptr()
        r.col_idx_dev = col_idx.data_ptr()
        r.precond = popts
        r.nsolves = k
        for i in range(k):
            r.vals_dev[i] = vals[i].data_ptr()
            r.b_dev[i] = bs[i].data_ptr()
            r.x_dev[i] = xs[i].data_ptr()
        _check(load().asm_server_submit(self._h, C.byref(r)))
        self._live[tag] = (row_ptr, col_idx, vals, bs, xs)

    def poll(self, max_done: int = 1024) -> list:
        """One scheduling round; returns the completions as dicts."""
        out = (Completion * max_done)()
        n = C.c_int32()
        _check(load().asm_server_poll(self._h, max_done, out, C.byref(n)))
        res = []
        for i in range(n.value):
            c = out[i]
            res.append({"tag": c.tag, "status": c.status, "solves": c.solves, "iters": c.iters,
                        "plan_cached": c.plan_cached, "rel_res_true": c.rel_res_true})
            self._live.pop(c.tag, None)
        return res

    def state(self) -> dict:
        st = ServerState()
        _check(load().asm_server_get_state(self._h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerState._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().asm_server_destroy(self._h)
            self._h = C.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
