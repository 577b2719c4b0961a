"""Thin ctypes binding of the mf C ABI (include/mf.h).

Argument marshalling only: every step of a product runs in libmf.so's HIP
kernels.  Torch is used for device memory (``tensor.data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  If the library is missing the
import fails; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# PyTorch for ROCm ships its own copy of the HIP runtime.  Loading torch before
# libmf.so makes the library bind to that copy, so the process holds ONE HIP
# runtime; loaded the other way round, the library would bring up a second
# runtime next to torch's, whose streams and events it cannot use.
import torch  # noqa: F401  (must precede the CDLL load below)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmf.so")

MF_OK = 0
MF_ERR_ARG = -1
MF_ERR_BRENT = -2
MF_ERR_SHAPE = -3
MF_ERR_NOMEM = -4
MF_ERR_HIP = -5
MF_ERR_UNSUPPORTED = -6
STATUS_NAMES = {0: "MF_OK", -1: "MF_ERR_ARG", -2: "MF_ERR_BRENT", -3: "MF_ERR_SHAPE", -4: "MF_ERR_NOMEM",
                -5: "MF_ERR_HIP", -6: "MF_ERR_UNSUPPORTED"}

MF_SCHED_FUSED = 1 << 16
MF_BATCH_PHASES = 0
MF_BATCH_PERSISTENT = 1
MF_F64 = 1
MF_F32 = 2
MF_LEAF_NATIVE = 0 << 8
MF_LEAF_F32 = 1 << 8
MF_LEAF_BF16 = 2 << 8
MF_LEAF_BF16X3 = 3 << 8
MF_W_ROWMAJOR_C = 0
MF_W_DEEPMIND_CT = 1

EXPORTED = ["mf_algo_from_uvw", "mf_algo_builtin", "mf_algo_compose", "mf_algo_rebase", "mf_algo_info",
            "mf_algo_get_uvw", "mf_algo_free", "mf_fastmm", "mf_classical_mm", "mf_workspace_bytes",
            "mf_fastmm_ws", "mf_fastmm_noalloc", "mf_last_error", "mf_phase_timing", "mf_phase_timing_read",
            "mf_batch_create", "mf_batch_create_form", "mf_batch_workspace_bytes", "mf_batch_run",
            "mf_batch_aborted", "mf_batch_tasks", "mf_batch_free", "mf_server_create", "mf_server_need_bytes", "mf_server_submit", "mf_server_replay",
            "mf_server_drain", "mf_server_stats", "mf_server_free", "mf_admission_simulate", "mf_fill_uniform",
            "mf_autotune_batch", "mf_plan_query", "mf_batch_phases", "mf_server_device_ms",
            "mf_server_submit_operands", "mf_server_device_interval", "mf_algo_from_uvw_rect",
            "mf_algo_classical", "mf_algo_concat", "mf_algo_shape", "mf_gemm"]


class ServerConfig(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int), ("hbm_budget", ctypes.c_size_t), ("allow_overtake", ctypes.c_int),
                ("depth_min_n_f64", ctypes.c_int64 * 4), ("depth_min_n_f32", ctypes.c_int64 * 4)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("levels_outer", ctypes.c_int), ("groups", ctypes.c_int),
                ("pre_stages", ctypes.c_int), ("post_stages", ctypes.c_int), ("leaf_m", ctypes.c_int64),
                ("products", ctypes.c_int64), ("gemm_flops", ctypes.c_double), ("pre_bytes", ctypes.c_double),
                ("post_bytes", ctypes.c_double), ("ws_bytes", ctypes.c_size_t)]


class MFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_12732_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    I64 = ctypes.c_int64
    DP = ctypes.POINTER(ctypes.c_double)
    LP = ctypes.POINTER(ctypes.c_int64)
    AP = ctypes.POINTER(P)
    sig = {
        "mf_algo_from_uvw": ([I, I, DP, DP, DP, I, AP], I),
        "mf_algo_builtin": ([ctypes.c_char_p, AP], I),
        "mf_algo_compose": ([P, P, AP], I),
        "mf_algo_rebase": ([P, LP, LP, LP, AP], I),
        "mf_algo_info": ([P] + [ctypes.POINTER(I)] * 5, I),
        "mf_algo_get_uvw": ([P, DP, DP, DP], I),
        "mf_algo_free": ([P], None),
        "mf_fastmm": ([P, I, I, P, P, P, I64, I, P], I),
        "mf_classical_mm": ([P, P, P, I64, I, P], I),
        "mf_workspace_bytes": ([P, I, I, I64, I, ctypes.POINTER(ctypes.c_size_t)], I),
        "mf_fastmm_ws": ([P, I, I, P, P, P, I64, I, P, ctypes.c_size_t, P], I),
        "mf_fastmm_noalloc": ([P, I, I, P, P, P, I64, I, P], I),
        "mf_algo_from_uvw_rect": ([I, I, I, I, DP, DP, DP, AP], I),
        "mf_algo_classical": ([I, I, I, AP], I),
        "mf_algo_concat": ([P, P, I, AP], I),
        "mf_algo_shape": ([P] + [ctypes.POINTER(I)] * 4, I),
        "mf_gemm": ([P, I, I, I64, I64, I64, ctypes.c_double, P, I64, P, I64, ctypes.c_double, P, I64, I, P], I),
        "mf_last_error": ([], ctypes.c_char_p),
        "mf_phase_timing": ([I], I),
        "mf_batch_create": ([I, LP, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(I), I, AP], I),
        "mf_batch_create_form": ([I, LP, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(I), I, I, AP], I),
        "mf_batch_workspace_bytes": ([P, ctypes.POINTER(ctypes.c_size_t)], I),
        "mf_batch_run": ([P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), P, ctypes.c_size_t, P], I),
        "mf_batch_aborted": ([P, ctypes.POINTER(I)], I),
        "mf_batch_tasks": ([P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(ctypes.c_int32)], I),
        "mf_batch_phases": ([P, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_int32)], I),
        "mf_batch_free": ([P], None),
        "mf_server_create": ([ctypes.POINTER(ServerConfig), P, AP], I),
        "mf_server_need_bytes": ([P, I64, I, ctypes.POINTER(ctypes.c_size_t)], I),
        "mf_server_submit": ([P, I64, I, ctypes.c_uint64, P, LP], I),
        "mf_server_replay": ([P, I, DP, LP, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_uint64)], I),
        "mf_server_drain": ([P], I),
        "mf_server_stats": ([P, LP, DP, DP, DP, LP, ctypes.POINTER(I)], I),
        "mf_server_free": ([P], None),
        "mf_server_device_ms": ([P, DP], I),
        "mf_server_device_interval": ([P, DP, DP], I),
        "mf_server_submit_operands": ([P, I64, I, P, P, P, LP], I),
        "mf_admission_simulate": ([I, DP, DP, ctypes.POINTER(ctypes.c_size_t), I, ctypes.c_size_t, I, DP, DP,
                                   ctypes.POINTER(ctypes.c_size_t)], I),
        "mf_fill_uniform": ([P, I64, I, ctypes.c_uint64, P], I),
        "mf_phase_timing_read": ([ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I)], I),
        "mf_plan_query": ([P, I, I, I64, I, ctypes.POINTER(PlanInfo)], I),
        "mf_autotune_batch": ([I, LP, I, ctypes.POINTER(P), I, I, ctypes.c_double, I, I, P, ctypes.POINTER(I), DP],
                              I),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


def _check(st: int):
    if st != MF_OK:
        raise MFError(st, lib.mf_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Algo:
    """Owning wrapper of an mf_algo handle."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        free = getattr(lib, "mf_algo_free", None) if lib is not None else None
        if h is not None and h.value and free is not None:
            free(h)
            self._h = ctypes.c_void_p(0)

    def info(self):
        vals = [ctypes.c_int() for _ in range(5)]
        _check(lib.mf_algo_info(self._h, *[ctypes.byref(v) for v in vals]))
        n0, R, nu, nv, nw = (v.value for v in vals)
        return {"n0": n0, "R": R, "nnz_u": nu, "nnz_v": nv, "nnz_w": nw}

    def shape(self):
        """(m0, k0, n0, R)."""
        vals = [ctypes.c_int() for _ in range(4)]
        _check(lib.mf_algo_shape(self._h, *[ctypes.byref(v) for v in vals]))
        return tuple(v.value for v in vals)

    def uvw(self):
        m0, k0, n0, R = self.shape()
        U = np.zeros((m0 * k0, R), dtype=np.float64)
        V = np.zeros((k0 * n0, R), dtype=np.float64)
        W = np.zeros((m0 * n0, R), dtype=np.float64)
        _check(lib.mf_algo_get_uvw(self._h, _dptr(U), _dptr(V), _dptr(W)))
        return U, V, W


def mf_algo_from_uvw(n0: int, U, V, W, w_convention: int = MF_W_ROWMAJOR_C) -> Algo:
    U = np.ascontiguousarray(U, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    if U.ndim != 2 or U.shape != V.shape or U.shape != W.shape:
        raise ValueError("U, V, W must be 2-d arrays of equal shape")
    out = ctypes.c_void_p()
    _check(lib.mf_algo_from_uvw(n0, U.shape[1], _dptr(U), _dptr(V), _dptr(W), w_convention, ctypes.byref(out)))
    return Algo(out.value)


def mf_algo_from_uvw_rect(m0: int, k0: int, n0: int, U, V, W) -> Algo:
    """<m0,k0,n0;R> from U (m0 k0 x R), V (k0 n0 x R), W (m0 n0 x R)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    V = np.ascontiguousarray(V, dtype=np.float64)
    W = np.ascontiguousarray(W, dtype=np.float64)
    R = U.shape[1]
    if U.shape != (m0 * k0, R) or V.shape != (k0 * n0, R) or W.shape != (m0 * n0, R):
        raise ValueError("U, V, W shapes do not match <m0,k0,n0;R>")
    out = ctypes.c_void_p()
    _check(lib.mf_algo_from_uvw_rect(m0, k0, n0, R, _dptr(U), _dptr(V), _dptr(W), ctypes.byref(out)))
    return Algo(out.value)


def mf_algo_classical(m0: int, k0: int, n0: int) -> Algo:
    out = ctypes.c_void_p()
    _check(lib.mf_algo_classical(m0, k0, n0, ctypes.byref(out)))
    return Algo(out.value)


AXIS = {"m": 0, "k": 1, "n": 2}


def mf_algo_concat(a: Algo, b: Algo, axis) -> Algo:
    """Direct sum along axis 'm' (0), 'k' (1) or 'n' (2)."""
    out = ctypes.c_void_p()
    _check(lib.mf_algo_concat(a.handle, b.handle, AXIS.get(axis, axis), ctypes.byref(out)))
    return Algo(out.value)


def mf_algo_builtin(name: str) -> Algo:
    out = ctypes.c_void_p()
    _check(lib.mf_algo_builtin(name.encode(), ctypes.byref(out)))
    return Algo(out.value)


def mf_algo_compose(outer: Algo, inner: Algo) -> Algo:
    out = ctypes.c_void_p()
    _check(lib.mf_algo_compose(outer.handle, inner.handle, ctypes.byref(out)))
    return Algo(out.value)


def mf_algo_rebase(a: Algo, X, Y, Z) -> Algo:
    mats = [np.ascontiguousarray(M, dtype=np.int64) for M in (X, Y, Z)]
    ptrs = [M.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) for M in mats]
    out = ctypes.c_void_p()
    _check(lib.mf_algo_rebase(a.handle, *ptrs, ctypes.byref(out)))
    return Algo(out.value)


def _dtype_code(t, leaf: int) -> int:
    import torch
    if t.dtype == torch.float64:
        return MF_F64 | leaf
    if t.dtype == torch.float32:
        return MF_F32 | leaf
    raise TypeError(f"unsupported tensor dtype {t.dtype}")


def _check_operands(A, B, C):
    for name, t in (("A", A), ("B", B), ("C", C)):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a device tensor")
        if t.dim() != 2 or t.shape[0] != t.shape[1] or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous square matrix")
    if not (A.shape == B.shape == C.shape) or not (A.dtype == B.dtype == C.dtype):
        raise ValueError("A, B, C must have equal shape and dtype")


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def mf_fastmm(algo: Algo, depth: int, cutoff: int, A, B, C, leaf: int = MF_LEAF_NATIVE, stream=None):
    """C = A B with ``depth`` levels of ``algo`` (torch device tensors)."""
    _check_operands(A, B, C)
    _check(lib.mf_fastmm(algo.handle, depth, cutoff, ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                         ctypes.c_void_p(C.data_ptr()), A.shape[0], _dtype_code(A, leaf), _stream(stream)))
    return C


def mf_fastmm_ws(algo: Algo, depth: int, cutoff: int, A, B, C, workspace, leaf: int = MF_LEAF_NATIVE,
                 stream=None):
    """As mf_fastmm with a caller-owned workspace tensor (any dtype)."""
    _check_operands(A, B, C)
    nbytes = workspace.numel() * workspace.element_size()
    _check(lib.mf_fastmm_ws(algo.handle, depth, cutoff, ctypes.c_void_p(A.data_ptr()),
                            ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(C.data_ptr()), A.shape[0],
                            _dtype_code(A, leaf), ctypes.c_void_p(workspace.data_ptr()), nbytes, _stream(stream)))
    return C


def mf_fastmm_noalloc(algo: Algo, depth: int, cutoff: int, A, B, C, leaf: int = MF_LEAF_NATIVE, stream=None):
    """As mf_fastmm, with descriptors and workspace in the library's fixed
    per-GPU scratch array (no device allocation in the call)."""
    _check_operands(A, B, C)
    _check(lib.mf_fastmm_noalloc(algo.handle, depth, cutoff, ctypes.c_void_p(A.data_ptr()),
                                 ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(C.data_ptr()), A.shape[0],
                                 _dtype_code(A, leaf), _stream(stream)))
    return C


def mf_gemm(algo, depth: int, cutoff: int, A, B, C, alpha: float = 1.0, beta: float = 0.0, stream=None,
            schedule: int = 0):
    """C = alpha A B + beta C for 2-d device tensors with unit column stride
    (row-major views; the row strides are the leading dimensions); schedule:
    0 or MF_SCHED_FUSED."""
    import torch
    for name, t in (("A", A), ("B", B), ("C", C)):
        if not t.is_cuda or t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
            raise ValueError(f"{name} must be a 2-d device tensor with unit column stride")
    if not (A.dtype == B.dtype == C.dtype) or A.dtype not in (torch.float64, torch.float32):
        raise ValueError("A, B, C must share dtype float64 or float32")
    M, K = A.shape
    K2, N = B.shape
    if K2 != K or tuple(C.shape) != (M, N):
        raise ValueError("shapes do not match C (M x N) = A (M x K) B (K x N)")
    code = (MF_F64 if A.dtype == torch.float64 else MF_F32) | schedule
    ld = lambda t: max(t.stride(0), t.shape[1])  # noqa: E731
    _check(lib.mf_gemm(algo.handle if algo is not None else None, depth, cutoff, M, N, K, float(alpha),
                       ctypes.c_void_p(A.data_ptr()), ld(A), ctypes.c_void_p(B.data_ptr()), ld(B), float(beta),
                       ctypes.c_void_p(C.data_ptr()), ld(C), code, _stream(stream)))
    return C


def mf_classical_mm(A, B, C, stream=None):
    """C = A B with the library's MFMA GEMM."""
    _check_operands(A, B, C)
    _check(lib.mf_classical_mm(ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                               ctypes.c_void_p(C.data_ptr()), A.shape[0], _dtype_code(A, 0), _stream(stream)))
    return C


def mf_workspace_bytes(algo: Algo, depth: int, cutoff: int, n: int, dtype_code: int = MF_F64) -> int:
    out = ctypes.c_size_t()
    _check(lib.mf_workspace_bytes(algo.handle, depth, cutoff, n, dtype_code, ctypes.byref(out)))
    return out.value


def mf_last_error() -> str:
    return lib.mf_last_error().decode()


def mf_phase_timing(enable: bool):
    """Enable or disable per-phase HIP-event timing of every call."""
    _check(lib.mf_phase_timing(1 if enable else 0))


def mf_phase_timing_read():
    """(summed ms of [pre-add, GEMM, post-add], number of calls) since the last read."""
    ms = (ctypes.c_double * 3)()
    calls = ctypes.c_int()
    _check(lib.mf_phase_timing_read(ms, ctypes.byref(calls)))
    return list(ms), calls.value


class Batch:
    """Owning wrapper of an mf_batch handle (keeps its algorithms alive)."""

    def __init__(self, handle: int, algos, sizes, dtype_code):
        self._h = ctypes.c_void_p(handle)
        self._algos = algos
        self.sizes = list(sizes)
        self.dtype_code = dtype_code

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        free = getattr(lib, "mf_batch_free", None) if lib is not None else None
        if h is not None and h.value and free is not None:
            free(h)
            self._h = ctypes.c_void_p(0)

    def workspace_bytes(self) -> int:
        out = ctypes.c_size_t()
        _check(lib.mf_batch_workspace_bytes(self._h, ctypes.byref(out)))
        return out.value

    def tasks(self):
        """(ntasks, nctr, int32 array [ntasks, 5]: type, instance, wait counter, wait value, done counter)."""
        nt, nc = ctypes.c_int(), ctypes.c_int()
        _check(lib.mf_batch_tasks(self._h, ctypes.byref(nt), ctypes.byref(nc), None))
        desc = np.zeros((nt.value, 5), dtype=np.int32)
        _check(lib.mf_batch_tasks(self._h, None, None, desc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return nt.value, nc.value, desc

    def phases(self):
        """int32 array [nphases, 3]: first task, end task, 1 for a GEMM phase."""
        npz = ctypes.c_int()
        _check(lib.mf_batch_phases(self._h, ctypes.byref(npz), None))
        desc = np.zeros((npz.value, 3), dtype=np.int32)
        _check(lib.mf_batch_phases(self._h, ctypes.byref(npz), desc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return desc

    def aborted(self) -> bool:
        flag = ctypes.c_int()
        _check(lib.mf_batch_aborted(self._h, ctypes.byref(flag)))
        return bool(flag.value)


def mf_batch_create(sizes, algos, depths, cutoffs, dtype_code: int = MF_F64, form: int = MF_BATCH_PHASES) -> Batch:
    """Plan a batch: algos[i] may be None where depths[i] == 0; form is
    MF_BATCH_PHASES (one launch per phase) or MF_BATCH_PERSISTENT (one launch)."""
    count = len(sizes)
    n_arr = (ctypes.c_int64 * count)(*sizes)
    a_arr = (ctypes.c_void_p * count)(*[(a.handle.value if a is not None else None) for a in algos])
    d_arr = (ctypes.c_int * count)(*depths)
    c_arr = (ctypes.c_int * count)(*cutoffs)
    out = ctypes.c_void_p()
    _check(lib.mf_batch_create_form(count, n_arr, a_arr, d_arr, c_arr, dtype_code, form, ctypes.byref(out)))
    return Batch(out.value, [a for a in algos if a is not None], sizes, dtype_code)


def mf_plan_query(algo, depth, cutoff, n, dtype_code=MF_F64) -> dict:
    """Shape and algorithmic cost of the plan of a request (host only)."""
    info = PlanInfo()
    _check(lib.mf_plan_query(algo.handle if algo is not None else None, depth, cutoff, n, dtype_code,
                             ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in PlanInfo._fields_}


def mf_autotune_batch(sizes, dtype_code, algos, max_depth, work_flops=2e11, max_copies=4096, reps=3, stream=None):
    """Tune (algorithm, depth) per size for the batched form.

    Returns (choices, ms): choices[i] is a (algo or None, depth) pair for
    sizes[i]; ms[i][c] is the device time per product of candidate c
    (classical first, then algos[j] at depths 1..max_depth), -1 if skipped.
    """
    k = len(sizes)
    ncand = 1 + len(algos) * max_depth
    n_arr = (ctypes.c_int64 * k)(*sizes)
    a_arr = (ctypes.c_void_p * max(1, len(algos)))(*[a.handle.value for a in algos])
    choice = (ctypes.c_int * k)()
    ms = (ctypes.c_double * (k * ncand))()
    _check(lib.mf_autotune_batch(k, n_arr, dtype_code, a_arr, len(algos), max_depth, float(work_flops), max_copies,
                                 reps, _stream(stream), choice, ms))
    out = []
    for i in range(k):
        c = choice[i]
        out.append((None, 0) if c == 0 else (algos[(c - 1) // max_depth], 1 + (c - 1) % max_depth))
    return out, [[ms[i * ncand + c] for c in range(ncand)] for i in range(k)]


def mf_batch_run(batch: Batch, As, Bs, Cs, workspace=None, stream=None):
    """Run a planned batch over lists of torch device tensors."""
    count = len(batch.sizes)
    if not (len(As) == len(Bs) == len(Cs) == count):
        raise ValueError("one A, B, C per instance")
    for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
        _check_operands(A, B, C)
        if A.shape[0] != batch.sizes[i]:
            raise ValueError(f"instance {i}: size {A.shape[0]} != planned {batch.sizes[i]}")
        if (_dtype_code(A, 0) & 0xff) != (batch.dtype_code & 0xff):
            raise TypeError(f"instance {i}: dtype does not match the batch")
    pa = (ctypes.c_void_p * count)(*[t.data_ptr() for t in As])
    pb = (ctypes.c_void_p * count)(*[t.data_ptr() for t in Bs])
    pc = (ctypes.c_void_p * count)(*[t.data_ptr() for t in Cs])
    ws = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
    nbytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib.mf_batch_run(batch.handle, pa, pb, pc, ws, nbytes, _stream(stream)))


class Server:
    """Owning wrapper of an mf_server (keeps its algorithm alive)."""

    def __init__(self, max_slots, hbm_budget, algo=None, depth_min_n_f64=(0, 0, 0, 0), depth_min_n_f32=(0, 0, 0, 0),
                 allow_overtake=False):
        cfg = ServerConfig()
        cfg.max_slots = max_slots
        cfg.hbm_budget = int(hbm_budget)
        cfg.allow_overtake = 1 if allow_overtake else 0
        for k in range(4):
            cfg.depth_min_n_f64[k] = int(depth_min_n_f64[k])
            cfg.depth_min_n_f32[k] = int(depth_min_n_f32[k])
        self._algo = algo
        out = ctypes.c_void_p()
        _check(lib.mf_server_create(ctypes.byref(cfg), algo.handle if algo is not None else None, ctypes.byref(out)))
        self._h = out

    def close(self):
        h = getattr(self, "_h", None)
        free = getattr(lib, "mf_server_free", None) if lib is not None else None
        if h is not None and h.value and free is not None:
            free(h)
            self._h = ctypes.c_void_p(0)

    __del__ = close

    def need_bytes(self, n, dtype_code):
        out = ctypes.c_size_t()
        _check(lib.mf_server_need_bytes(self._h, n, dtype_code, ctypes.byref(out)))
        return out.value

    def submit(self, n, dtype_code, seed, host_out=None):
        """host_out: pinned torch CPU tensor of n*n elements (or None)."""
        rid = ctypes.c_int64()
        ptr = ctypes.c_void_p(host_out.data_ptr()) if host_out is not None else None
        _check(lib.mf_server_submit(self._h, n, dtype_code, seed, ptr, ctypes.byref(rid)))
        return rid.value

    def submit_operands(self, A, B, C):
        """C = A B on caller-owned torch device tensors (kept alive until drained)."""
        _check_operands(A, B, C)
        rid = ctypes.c_int64()
        _check(lib.mf_server_submit_operands(self._h, A.shape[0], _dtype_code(A, 0), ctypes.c_void_p(A.data_ptr()),
                                             ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(C.data_ptr()),
                                             ctypes.byref(rid)))
        self._keep = getattr(self, "_keep", []) + [(A, B, C)]
        return rid.value

    def replay(self, t_arrive, ns, dtype_codes, seeds):
        k = len(ns)
        t = np.ascontiguousarray(t_arrive, dtype=np.float64)
        nn = np.ascontiguousarray(ns, dtype=np.int64)
        dd = np.ascontiguousarray(dtype_codes, dtype=np.int32)
        ss = np.ascontiguousarray(seeds, dtype=np.uint64)
        _check(lib.mf_server_replay(self._h, k, _dptr(t), nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    dd.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                    ss.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))

    def drain(self):
        _check(lib.mf_server_drain(self._h))

    def stats(self):
        cnt = ctypes.c_int64()
        _check(lib.mf_server_stats(self._h, ctypes.byref(cnt), None, None, None, None, None))
        c = cnt.value
        ta, tm, td = (np.zeros(c) for _ in range(3))
        nn = np.zeros(c, dtype=np.int64)
        dp = np.zeros(c, dtype=np.int32)
        _check(lib.mf_server_stats(self._h, ctypes.byref(cnt), _dptr(ta), _dptr(tm), _dptr(td),
                                   nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   dp.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        dev = np.zeros(c)
        _check(lib.mf_server_device_ms(self._h, _dptr(dev)))
        d0, d1 = np.zeros(c), np.zeros(c)
        _check(lib.mf_server_device_interval(self._h, _dptr(d0), _dptr(d1)))
        return {"t_arrive": ta, "t_admit": tm, "t_done": td, "n": nn, "depth": dp, "device_ms": dev,
                "device_start_ms": d0, "device_end_ms": d1}


def mf_admission_simulate(t_arrive, service, need, slots, budget, allow_overtake=False):
    k = len(t_arrive)
    t = np.ascontiguousarray(t_arrive, dtype=np.float64)
    sv = np.ascontiguousarray(service, dtype=np.float64)
    nd = (ctypes.c_size_t * k)(*[int(x) for x in need])
    ta = np.zeros(k)
    td = np.zeros(k)
    peak = ctypes.c_size_t()
    _check(lib.mf_admission_simulate(k, _dptr(t), _dptr(sv), nd, slots, int(budget), 1 if allow_overtake else 0,
                                     _dptr(ta), _dptr(td), ctypes.byref(peak)))
    return ta, td, peak.value


def mf_fill_uniform(t, seed, stream=None):
    """Fill a device tensor (float64 or float32) with the serving generator."""
    code = _dtype_code(t, 0)
    _check(lib.mf_fill_uniform(ctypes.c_void_p(t.data_ptr()), t.numel(), code, seed, _stream(stream)))
    return t
