"""Python binding of libpbicgstab.so (MI355X exact-reduction pipelined BiCGStab).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides device memory and the current stream.  The binding raises if
the compiled library is missing -- there is no fallback path.

Functions mirror the C-ABI in include/pbicgstab.h:
``csr_spmv``, ``csr_spmv_f32``, ``exdot``, ``exdot_config``, ``pbcg_phase_a``,
``pbcg_phase_b``, ``pbicgstab_solve``; ``CSR`` wraps device CSR tensors and
``solve`` is the convenience driver (allocates the workspace with torch).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbicgstab.so")

OK, NOT_CONVERGED, BREAKDOWN, STAGNATED = 0, 1, 2, 3
ERR_INVALID, ERR_HIP, ERR_NONFINITE, ERR_WORKSPACE = -1, -2, -3, -4
F64, F32 = 0, 1
ALG_PBICGSTAB, ALG_BICGSTAB = 0, 1
PREC_FP64, PREC_FP32_IR, PREC_FP32_MATRIX = 0, 1, 2
SPMV_SEQ, SPMV_VECTOR, SPMV_WAVE = 0, 1, 2
DOTS_EXACT, DOTS_PLAIN = 0, 1
LAYOUT_AUTO, LAYOUT_CSR, LAYOUT_SORTED, LAYOUT_SLICED = 0, 1, 2, 3

_P = ctypes.c_void_p


class PbcgCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("val_type", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", _P), ("col_idx", _P), ("val", _P)]


class PbcgOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("alg", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("max_outer", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("M", ctypes.POINTER(PbcgCsr)), ("fallback", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("history", _P), ("r_out", _P),
                ("batch", ctypes.c_int32), ("stall_window", ctypes.c_int32),
                ("spmv_kind", ctypes.c_int32), ("trace", ctypes.c_int32),
                ("dots", ctypes.c_int32), ("rr_period", ctypes.c_int32),
                ("true_every", ctypes.c_int32), ("true_history_len", ctypes.c_int32),
                ("true_history", ctypes.c_void_p), ("layout", ctypes.c_int32),
                ("kernel_events_len", ctypes.c_int32), ("kernel_events", ctypes.POINTER(ctypes.c_void_p)),
                ("exact_rows", ctypes.c_int32)]


class PbcgInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("outer_iterations", ctypes.c_int32), ("true_checks", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("sliced", ctypes.c_int32),
                ("true_relres", ctypes.c_double), ("rec_relres", ctypes.c_double),
                ("seconds", ctypes.c_double), ("sliced_entries", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PbcgSliced(ctypes.Structure):
    _fields_ = [("entries", ctypes.c_int64), ("slice_off", _P), ("col", _P), ("val", _P)]


class PbcgVectors(ctypes.Structure):
    _fields_ = [(k, _P) for k in ("x", "r", "rhat", "w", "t", "p", "s", "z", "q", "y", "v")]


EXPORTS = [
    "csr_spmv", "csr_spmv_exact", "csr_spmv_config", "csr_spmv_f32", "csr_jacobi", "csr_slice_workspace_bytes", "csr_slice",
    "csr_spmv_sliced", "csr_spmv_f32_sliced", "exdot_workspace_bytes", "exdot", "exdot_config",
    "exdot_noalloc_scratch_bytes", "exdot_noalloc", "plain_dot_workspace_bytes", "plain_dot",
    "pbcg_phase_workspace_bytes", "pbcg_phase_a", "pbcg_phase_b", "pbicgstab_workspace_bytes",
    "pbicgstab_solve", "pbcg_default_opts", "pbcg_status_string", "pbcg_abi_version",
    "spai_param_count", "spai_workspace_bytes", "spai_features", "spai_forward", "spai_infer_bf16",
    "spai_probe_product", "spai_loss_grad", "spai_adam", "spai_train_step", "spai_probe_column_workspace_bytes",
    "spai_probe_column",
]

_lib = None


def lib():
    """Load libpbicgstab.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2404_13216_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, sz, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    CP = ctypes.POINTER(PbcgCsr)
    sig = {
        "csr_spmv": (ctypes.c_int, [CP, _P, _P, _P]),
        "csr_spmv_exact": (ctypes.c_int, [CP, _P, _P, _P]),
        "csr_spmv_config": (ctypes.c_int, [CP, _P, _P, i32, _P]),
        "csr_spmv_f32": (ctypes.c_int, [CP, _P, _P, _P]),
        "csr_jacobi": (ctypes.c_int, [CP, _P, i32, _P]),
        "csr_slice_workspace_bytes": (sz, [i32, i64]),
        "csr_slice": (ctypes.c_int, [CP, ctypes.POINTER(PbcgSliced), _P, sz, _P]),
        "csr_spmv_sliced": (ctypes.c_int, [CP, ctypes.POINTER(PbcgSliced), _P, _P, _P]),
        "csr_spmv_f32_sliced": (ctypes.c_int, [CP, ctypes.POINTER(PbcgSliced), _P, _P, _P]),
        "exdot_workspace_bytes": (sz, [i64]),
        "exdot": (ctypes.c_int, [i64, _P, _P, _P, _P, sz, _P]),
        "exdot_config": (ctypes.c_int, [i64, _P, _P, _P, i32, i32, i32, _P, sz, _P]),
        "exdot_noalloc_scratch_bytes": (sz, []),
        "exdot_noalloc": (ctypes.c_int, [i64, _P, _P, _P, _P]),
        "plain_dot_workspace_bytes": (sz, [i64]),
        "plain_dot": (ctypes.c_int, [i64, _P, _P, i32, _P, _P, sz, _P]),
        "pbcg_phase_workspace_bytes": (sz, [i32]),
        "pbcg_phase_a": (ctypes.c_int, [i32, ctypes.POINTER(PbcgVectors), _P, i32, _P, _P, sz, _P]),
        "pbcg_phase_b": (ctypes.c_int, [i32, ctypes.POINTER(PbcgVectors), _P, _P, _P, sz, _P]),
        "pbicgstab_workspace_bytes": (sz, [i32, i64, ctypes.POINTER(PbcgOpts)]),
        "pbicgstab_solve": (ctypes.c_int, [CP, _P, _P, ctypes.POINTER(PbcgOpts), ctypes.POINTER(PbcgInfo),
                                           _P, sz, _P]),
        "pbcg_default_opts": (None, [ctypes.POINTER(PbcgOpts)]),
        "pbcg_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "pbcg_abi_version": (ctypes.c_int, []),
        "spai_param_count": (ctypes.c_int, []),
        "spai_workspace_bytes": (sz, [i32, i64, i32]),
        "spai_features": (ctypes.c_int, [CP, _P, _P, _P, _P, sz, _P]),
        "spai_forward": (ctypes.c_int, [i64, _P, _P, _P, _P, _P, _P, _P, _P]),
        "spai_infer_bf16": (ctypes.c_int, [i64, _P, _P, _P, _P, _P, _P]),
        "spai_probe_product": (ctypes.c_int, [CP, _P, i32, _P, _P]),
        "spai_probe_column_workspace_bytes": (sz, [i32]),
        "spai_probe_column": (ctypes.c_int, [i32, _P, _P, _P, sz, _P]),
        "spai_loss_grad": (ctypes.c_int, [CP, _P, _P, _P, _P, _P, _P, i32, _P, _P, _P, _P, sz, _P]),
        "spai_adam": (ctypes.c_int, [_P, _P, _P, _P, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, _P]),
        "spai_train_step": (ctypes.c_int, [CP, _P, _P, _P, _P, _P, i32, _P, _P, _P, i32,
                                           ctypes.POINTER(ctypes.c_float), _P, _P, sz, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def status_string(code: int) -> str:
    return lib().pbcg_status_string(int(code)).decode()


class LibError(RuntimeError):
    pass


def _check(code: int, what: str):
    if code < 0:
        raise LibError(f"{what}: {status_string(code)} ({code})")
    return code


# --------------------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes: int, device):
    torch = _torch()
    # 256-byte aligned by the caching allocator (allocations are 512-byte aligned)
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class CSR:
    """Device CSR (int32 row_ptr / col_idx, float64 or float32 values)."""

    def __init__(self, row_ptr, col_idx, val, n=None):
        torch = _torch()
        self.row_ptr = row_ptr.to(torch.int32).contiguous()
        self.col_idx = col_idx.to(torch.int32).contiguous()
        self.val = val.contiguous()
        assert self.val.dtype in (torch.float64, torch.float32)
        self.n = int(n if n is not None else self.row_ptr.numel() - 1)
        self.nnz = int(self.col_idx.numel())
        self._c = PbcgCsr(self.n, F64 if self.val.dtype == torch.float64 else F32, self.nnz,
                          self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.val.data_ptr())

    @classmethod
    def from_host(cls, A, device="cuda", dtype=None):
        """From a synthgen.CSR (numpy arrays)."""
        torch = _torch()
        val = torch.from_numpy(np.ascontiguousarray(A.val))
        if dtype is not None:
            val = val.to(dtype)
        return cls(torch.from_numpy(A.row_ptr).to(device), torch.from_numpy(A.col_idx).to(device),
                   val.to(device), A.n)

    def with_values(self, val):
        return CSR(self.row_ptr, self.col_idx, val, self.n)

    @property
    def c(self):
        return ctypes.byref(self._c)


class SlicedCSR:
    """Sliced copy of a device CSR (csr_slice); `built` is False when its padding is
    too large, and the CSR form is then the one to use."""

    def __init__(self, A: CSR):
        self.A = A
        self.ws = _workspace(lib().csr_slice_workspace_bytes(A.n, A.nnz), A.val.device)
        self._c = PbcgSliced()
        _check(lib().csr_slice(A.c, ctypes.byref(self._c), _ptr(self.ws), self.ws.numel(), _stream()),
               "csr_slice")

    @property
    def built(self) -> bool:
        return bool(self._c.slice_off)

    @property
    def entries(self) -> int:
        return int(self._c.entries)

    @property
    def c(self):
        return ctypes.byref(self._c)


def csr_spmv_sliced(S: SlicedCSR, x, y=None):
    torch = _torch()
    if y is None:
        y = torch.empty(S.A.n, dtype=torch.float64, device=x.device)
    _check(lib().csr_spmv_sliced(S.A.c, S.c, _ptr(x), _ptr(y), _stream()), "csr_spmv_sliced")
    return y


def csr_spmv_f32_sliced(S: SlicedCSR, x, y=None):
    torch = _torch()
    if y is None:
        y = torch.empty(S.A.n, dtype=torch.float32, device=x.device)
    _check(lib().csr_spmv_f32_sliced(S.A.c, S.c, _ptr(x), _ptr(y), _stream()), "csr_spmv_f32_sliced")
    return y


def csr_spmv(A: CSR, x, y=None, kind: int | None = None):
    torch = _torch()
    if y is None:
        y = torch.empty(A.n, dtype=torch.float64, device=x.device)
    if kind is None:
        _check(lib().csr_spmv(A.c, _ptr(x), _ptr(y), _stream()), "csr_spmv")
    else:
        _check(lib().csr_spmv_config(A.c, _ptr(x), _ptr(y), int(kind), _stream()), "csr_spmv_config")
    return y


def csr_spmv_exact(A: CSR, x, y=None):
    """y = A x with every row summed exactly and rounded once."""
    torch = _torch()
    if y is None:
        y = torch.empty(A.n, dtype=torch.float64, device=x.device)
    _check(lib().csr_spmv_exact(A.c, _ptr(x), _ptr(y), _stream()), "csr_spmv_exact")
    return y


def csr_spmv_f32(A: CSR, x, y=None):
    torch = _torch()
    if y is None:
        y = torch.empty(A.n, dtype=torch.float32, device=x.device)
    _check(lib().csr_spmv_f32(A.c, _ptr(x), _ptr(y), _stream()), "csr_spmv_f32")
    return y


def csr_validate(A) -> None:
    """Host-side structural check of a CSR (a synthgen.CSR or a device CSR, copied to the
    host): row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz < 2^31; columns in [0, n)
    and strictly ascending within every row.  Raises ValueError.  The kernels take the
    column ranges on trust; this is the check to run on untrusted input."""
    rp = A.row_ptr.cpu().numpy() if hasattr(A.row_ptr, "cpu") else np.asarray(A.row_ptr)
    ci = A.col_idx.cpu().numpy() if hasattr(A.col_idx, "cpu") else np.asarray(A.col_idx)
    n = int(A.n)
    rp = rp.astype(np.int64)
    ci = ci.astype(np.int64)
    if rp.shape != (n + 1,) or rp[0] != 0:
        raise ValueError("row_ptr must have n + 1 entries starting at 0")
    if np.any(np.diff(rp) < 0):
        raise ValueError("row_ptr must be non-decreasing")
    if rp[-1] != ci.size or ci.size >= 2 ** 31:
        raise ValueError("row_ptr[n] must equal nnz (< 2^31)")
    if ci.size and (ci.min() < 0 or ci.max() >= n):
        raise ValueError("column index out of range")
    if ci.size > 1:
        same_row = np.repeat(np.arange(n), np.diff(rp))
        d = np.diff(ci)
        if np.any((d <= 0) & (same_row[1:] == same_row[:-1])):
            raise ValueError("columns must be strictly ascending within a row")


def jacobi(A: CSR, dtype=None) -> CSR:
    """Diagonal right preconditioner M = diag(1/a_ii) as a CSR with one entry per row;
    the values come from csr_jacobi (FP64 reciprocal rounded once to `dtype`)."""
    torch = _torch()
    dtype = torch.float64 if dtype is None else dtype
    dev = A.val.device
    m = torch.empty(A.n, dtype=dtype, device=dev)
    _check(lib().csr_jacobi(A.c, _ptr(m), F64 if dtype == torch.float64 else F32, _stream()), "csr_jacobi")
    idx = torch.arange(A.n + 1, dtype=torch.int32, device=dev)
    return CSR(idx, idx[:-1].clone(), m, n=A.n)


def exdot(x, y, out=None, ws=None):
    torch = _torch()
    n = x.numel()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    nb = lib().exdot_workspace_bytes(n)
    if ws is None:
        ws = _workspace(nb, x.device)
    _check(lib().exdot(n, _ptr(x), _ptr(y), _ptr(out), _ptr(ws), ws.numel(), _stream()), "exdot")
    return out


def exdot_noalloc(x, y, out):
    """exdot without a workspace: the library's static scratch array holds the records.
    `out` is a caller-owned one-element float64 device tensor (nothing is allocated)."""
    _check(lib().exdot_noalloc(x.numel(), _ptr(x), _ptr(y), _ptr(out), _stream()), "exdot_noalloc")
    return out


def plain_dot(x, y, out=None, ws=None):
    """Plain dot in the library's fixed reduction tree (float32 or float64 vectors)."""
    torch = _torch()
    n = x.numel()
    if out is None:
        out = torch.empty(1, dtype=x.dtype, device=x.device)
    if ws is None:
        ws = _workspace(lib().plain_dot_workspace_bytes(n), x.device)
    dt = F64 if x.dtype == torch.float64 else F32
    _check(lib().plain_dot(n, _ptr(x), _ptr(y), dt, _ptr(out), _ptr(ws), ws.numel(), _stream()), "plain_dot")
    return out


def exdot_config(x, y, grid, block, k, out=None, ws=None):
    torch = _torch()
    n = x.numel()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    nb = lib().exdot_workspace_bytes(n)
    if ws is None:
        ws = _workspace(nb, x.device)
    _check(lib().exdot_config(n, _ptr(x), _ptr(y), _ptr(out), int(grid), int(block), int(k), _ptr(ws),
                              ws.numel(), _stream()), "exdot_config")
    return out


def _vectors(V: dict) -> PbcgVectors:
    return PbcgVectors(*[V[k].data_ptr() if V.get(k) is not None else None
                         for k in ("x", "r", "rhat", "w", "t", "p", "s", "z", "q", "y", "v")])


def pbcg_phase_a(V: dict, scal, first: bool, dots_out=None, ws=None):
    torch = _torch()
    n = V["r"].numel()
    if dots_out is None:
        dots_out = torch.empty(4, dtype=torch.float64, device=V["r"].device)
    if ws is None:
        ws = _workspace(lib().pbcg_phase_workspace_bytes(n), V["r"].device)
    vs = _vectors(V)
    _check(lib().pbcg_phase_a(n, ctypes.byref(vs), _ptr(scal), int(bool(first)), _ptr(dots_out), _ptr(ws),
                              ws.numel(), _stream()), "pbcg_phase_a")
    return dots_out


def pbcg_phase_b(V: dict, scal, dots_out=None, ws=None):
    torch = _torch()
    n = V["r"].numel()
    if dots_out is None:
        dots_out = torch.empty(3, dtype=torch.float64, device=V["r"].device)
    if ws is None:
        ws = _workspace(lib().pbcg_phase_workspace_bytes(n), V["r"].device)
    vs = _vectors(V)
    _check(lib().pbcg_phase_b(n, ctypes.byref(vs), _ptr(scal), _ptr(dots_out), _ptr(ws), ws.numel(),
                              _stream()), "pbcg_phase_b")
    return dots_out


def default_opts(**kw) -> PbcgOpts:
    o = PbcgOpts()
    lib().pbcg_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Solver:
    """Holds a workspace for repeated solves with one matrix and option set."""

    KERNELS = ("phase_a", "spmv_az", "phase_b", "spmv_aw")

    def __init__(self, A: CSR, M: CSR | None = None, history: int = 0, kernel_events: int = 0, **opts):
        torch = _torch()
        self.A, self.M = A, M
        self.opts = default_opts(**opts)
        # measurement: start/end events of the four kernels of iterations 1..kernel_events
        # (FP64 p-BiCGStab, exact dots, no M), stamped by the kernels' own dispatches
        self._events = []
        if kernel_events:
            self._events = [torch.cuda.Event(enable_timing=True) for _ in range(8 * kernel_events)]
            for e in self._events:      # creates the HIP events
                e.record()
            torch.cuda.synchronize()
            self._ev_ptrs = (ctypes.c_void_p * len(self._events))(*[e.cuda_event for e in self._events])
            self.opts.kernel_events = ctypes.cast(self._ev_ptrs, ctypes.POINTER(ctypes.c_void_p))
            self.opts.kernel_events_len = len(self._events)
        self._M_ref = M
        if M is not None:
            self.opts.M = ctypes.pointer(M._c)
        self.history = None
        if history:
            self.history = torch.full((history,), float("nan"), dtype=torch.float64, device=A.val.device)
            self.opts.history = self.history.data_ptr()
            self.opts.history_len = history
        self.true_history = None
        if self.opts.true_every > 0:
            cap = max(self.opts.max_iter // self.opts.true_every, 1)
            self.true_history = torch.full((cap,), float("nan"), dtype=torch.float64, device=A.val.device)
            self.opts.true_history = self.true_history.data_ptr()
            self.opts.true_history_len = cap
        nb = lib().pbicgstab_workspace_bytes(A.n, A.nnz, ctypes.byref(self.opts))
        self.ws = _workspace(nb, A.val.device)

    def kernel_times(self):
        """Durations (seconds) of the timed kernels of the last solve, per kernel role."""
        torch = _torch()
        torch.cuda.synchronize()
        ev = self._events
        out = {k: [] for k in self.KERNELS}
        for j in range(len(ev) // 8):
            for k, name in enumerate(self.KERNELS):
                out[name].append(ev[8 * j + 2 * k].elapsed_time(ev[8 * j + 2 * k + 1]) / 1e3)
        return out

    def solve(self, b, x=None, r_out=None):
        torch = _torch()
        if x is None:
            x = torch.zeros(self.A.n, dtype=torch.float64, device=b.device)
        self.opts.r_out = r_out.data_ptr() if r_out is not None else None
        info = PbcgInfo()
        code = lib().pbicgstab_solve(self.A.c, _ptr(b), _ptr(x), ctypes.byref(self.opts), ctypes.byref(info),
                                     _ptr(self.ws), self.ws.numel(), _stream())
        if code in (ERR_INVALID, ERR_HIP, ERR_WORKSPACE):
            raise LibError(f"pbicgstab_solve: {status_string(code)} ({code})")
        return x, info.as_dict()


def solve(A: CSR, b, x0=None, M: CSR | None = None, history: int = 0, **opts):
    """Solve A x = b on the GPU; returns (x, info dict)."""
    s = Solver(A, M=M, history=history, **opts)
    x = x0.clone() if x0 is not None else None
    x, info = s.solve(b, x)
    if history:
        info["history"] = s.history[: info["iterations"]].cpu().numpy()
    if s.true_history is not None:
        th = s.true_history.cpu().numpy()
        info["true_history"] = th[~np.isnan(th)]
    return x, info


def read_matrix_market(src):
    """Square coordinate Matrix Market file -> host CSR (see paper_2404_13216_amd.mtx)."""
    from .mtx import read_matrix_market as _r
    return _r(src)
