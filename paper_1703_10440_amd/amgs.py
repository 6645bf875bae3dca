"""Thin ctypes binding of the HIP library ``libamgs.so`` (C ABI in
``include/amgs.h``).

Functions named ``amgs_*`` mirror the C entry points one to one (argument
marshalling only).  ``qr_csr`` / ``qr_dense`` / ``BatchPlan`` are
conveniences that allocate outputs and workspace with torch (device memory
and streams only) and call those entry points; every arithmetic step runs in
the library's kernels.  If the library is missing this module raises: there
is no other implementation to fall back to.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libamgs.so")

VARIANTS = {"naive": 0, "ha": 1, "hp": 2}
PRECISIONS = {"fp64": 0, "fp32": 1}
STATUS = {0: "ok", -1: "invalid argument", -2: "workspace too small", -3: "HIP error",
          -4: "unsupported"}


class AmgsError(RuntimeError):
    pass


class Opts(C.Structure):
    _fields_ = [("reorth", C.c_int32), ("panel", C.c_int32), ("cgs", C.c_int32),
                ("first", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("mv_calls", C.c_int64), ("mv_columns", C.c_int64),
                ("kernel_launches", C.c_int64), ("sweep_launches", C.c_int64),
                ("sweep_bytes", C.c_double), ("mv_bytes", C.c_double),
                ("block_sweep_launches", C.c_int64), ("block_sweep_bytes", C.c_double)]


class BatchDesc(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("vals", C.c_void_p),
                ("Z", C.c_void_p), ("ldz", C.c_int64), ("Q", C.c_void_p), ("ldq", C.c_int64),
                ("R", C.c_void_p), ("ldr", C.c_int64)]


_lib = None

# (name, restype, argtypes) of every exported entry point
_vp, _i64, _i32, _sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
_SIGS = [
    ("amgs_create", C.c_int, [C.POINTER(_vp), C.c_int]),
    ("amgs_destroy", C.c_int, [_vp]),
    ("amgs_workspace_bytes", _sz, [_vp, _i64, _i64, _i32, C.c_int, C.c_int, _i32,
                                   C.POINTER(Opts)]),
    ("amgs_qr_csr", C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                              _i64, _vp, _i64, C.c_int, C.c_int, C.POINTER(Opts), _vp, _sz, _vp,
                              _vp]),
    ("amgs_qr_csr_static", C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _i64, _vp, _i64, _vp,
                                     _i64, _vp, _i64, _vp, _i64, C.c_int, C.c_int,
                                     C.POINTER(Opts), _vp, _vp]),
    ("amgs_qr_dense", C.c_int, [_vp, _i64, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                _i64, C.c_int, C.c_int, C.POINTER(Opts), _vp, _sz, _vp, _vp]),
    ("amgs_csr_check", C.c_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp]),
    ("amgs_batch_plan_create", C.c_int, [_vp, _i32, C.POINTER(_i64), C.POINTER(_i64), C.c_int,
                                         C.c_int, C.POINTER(Opts), _i32, C.POINTER(_vp)]),
    ("amgs_batch_plan_destroy", C.c_int, [_vp]),
    ("amgs_batch_workspace_bytes", _sz, [_vp]),
    ("amgs_qr_batched", C.c_int, [_vp, _vp, _vp, _sz, _vp, _vp]),
    ("amgs_batch_plan_tiles", _i32, [_vp, C.POINTER(_i32), _i32]),
    ("amgs_get_stats", C.c_int, [_vp, C.POINTER(Stats)]),
    ("amgs_status_string", C.c_char_p, [C.c_int]),
    ("amgs_profile_enable", C.c_int, [_vp, _i32]),
    ("amgs_profile_read", C.c_int, [_vp, _i32, C.POINTER(C.c_double), C.POINTER(_i64)]),
    ("amgs_profile_reset", C.c_int, [_vp]),
]
EXPORTS = [s[0] for s in _SIGS]


def load(path: Optional[str] = None):
    """Load libamgs.so (built by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    # AMGS_LIB_PATH selects another build of the same library (tuning runs)
    p = path or os.environ.get("AMGS_LIB_PATH") or LIB_PATH
    if not os.path.exists(p):
        raise AmgsError(f"HIP library not built: {p} is missing (run __graft_entry__.build())")
    lib = C.CDLL(p)
    for name, res, args in _SIGS:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(status: int, what: str):
    if status != 0:
        raise AmgsError(f"{what}: {STATUS.get(status, status)}")


# ----------------------------------------------------------- raw entry points
def amgs_create(device: int = 0) -> int:
    h = _vp()
    _check(load().amgs_create(C.byref(h), device), "amgs_create")
    return h.value


def amgs_destroy(h: int) -> int:
    return load().amgs_destroy(h)


def amgs_workspace_bytes(h, m, n, is_dense, variant, precision, P_given, opts=None) -> int:
    return int(load().amgs_workspace_bytes(h, m, n, is_dense, variant, precision, P_given,
                                            C.byref(opts) if opts is not None else None))


def amgs_qr_csr(*args) -> int:
    return load().amgs_qr_csr(*args)


def amgs_qr_csr_static(*args) -> int:
    return load().amgs_qr_csr_static(*args)


def amgs_qr_dense(*args) -> int:
    return load().amgs_qr_dense(*args)


def amgs_csr_check(*args) -> int:
    return load().amgs_csr_check(*args)


def amgs_get_stats(h) -> Stats:
    s = Stats()
    _check(load().amgs_get_stats(h, C.byref(s)), "amgs_get_stats")
    return s


def amgs_status_string(s: int) -> str:
    return load().amgs_status_string(s).decode()


def amgs_profile_enable(h, on: int) -> int:
    return load().amgs_profile_enable(h, on)


def amgs_profile_read(h, category: int):
    ms, n = C.c_double(), _i64()
    _check(load().amgs_profile_read(h, category, C.byref(ms), C.byref(n)), "amgs_profile_read")
    return ms.value, n.value


def amgs_profile_reset(h) -> int:
    return load().amgs_profile_reset(h)


# --------------------------------------------------------------- conveniences
_handles = {}


def handle(device: int = 0) -> int:
    if device not in _handles:
        _handles[device] = amgs_create(device)
    return _handles[device]


def _torch():
    import torch
    return torch


def colmajor(t, dtype=None):
    """Return an (m, n) column-major (stride (1, m)) device copy/view of t."""
    torch = _torch()
    if dtype is not None and t.dtype != dtype:
        t = t.to(dtype)
    if t.dim() == 1:
        t = t[:, None]
    m, n = t.shape
    if t.stride(0) == 1 and t.stride(1) >= max(m, 1):
        return t
    return t.t().contiguous().t()


def empty_colmajor(m, n, dtype, device):
    torch = _torch()
    return torch.empty((n, m), dtype=dtype, device=device).t()


@dataclass
class QRResult:
    Q: object       # (m, n) column-major device tensor
    R: object       # (n, n) column-major float64 device tensor
    P: object       # (m, n) column-major device tensor (= A Q), or None
    info: object    # int32 device tensor with one entry
    stats: Stats


def _check_out(t, name, rows, cols, dtype, device):
    """A caller's output buffer must be exactly what the kernels write: the C
    ABI takes a bare pointer and a leading dimension and cannot check it."""
    if not (t.dim() == 2 and tuple(t.shape) == (rows, cols)):
        raise ValueError(f"{name} must be {rows} x {cols}, got {tuple(t.shape)}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if rows > 0 and cols > 0 and not (t.stride(0) == 1 and (cols == 1 or t.stride(1) >= rows)):
        raise ValueError(f"{name} must be column-major (stride(0) == 1, stride(1) >= {rows}), "
                         f"got strides {t.stride()}")


@contextlib.contextmanager
def _on_stream(stream, device, caller_tensors):
    """Run a call's preparation and launches on `stream` (None: torch's
    current stream; else a torch stream or a raw hipStream_t handle).  A
    stream other than the current one first waits for the current stream, so
    the caller's inputs are complete; the conversions, outputs and workspace
    the binding allocates are then made on that stream, and the caller's own
    tensors are recorded as in use by it, so the caching allocator does not
    hand their memory out again before the stream has finished with it.
    Yields the raw stream handle to pass to the library."""
    torch = _torch()
    cur = torch.cuda.current_stream(device)
    if stream is None:
        yield cur.cuda_stream
        return
    if not isinstance(stream, torch.cuda.Stream):
        stream = torch.cuda.ExternalStream(int(stream), device=device)
    if stream.cuda_stream == cur.cuda_stream:
        yield cur.cuda_stream
        return
    stream.wait_stream(cur)
    with torch.cuda.stream(stream):
        yield stream.cuda_stream
    for t in caller_tensors:
        if t is not None and t.is_cuda:
            t.record_stream(stream)


def _workspace(work, wb, device):
    """The caller's workspace (its size in bytes is what the library checks),
    or a new one of wb bytes."""
    if work is None:
        return _torch().empty(max(wb, 1), dtype=_torch().uint8, device=device)
    if not work.is_contiguous():
        raise ValueError("work must be contiguous")
    if work.device != device:
        raise ValueError(f"work must be on {device}, got {work.device}")
    return work


def _prep(Z, precision, device, Q, P, return_p, R=None):
    torch = _torch()
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}, got {precision!r}")
    dt = torch.float64 if precision == "fp64" else torch.float32
    Zc = colmajor(Z.to(device), dt)
    m, n = Zc.shape
    device = Zc.device
    for t, name, rows, cols, tdt in ((Q, "Q", m, n, dt), (P, "P", m, n, dt),
                                     (R, "R", n, n, torch.float64)):
        if t is not None:
            _check_out(t, name, rows, cols, tdt, device)
    Qc = Q if Q is not None else empty_colmajor(m, n, dt, device)
    R = R if R is not None else empty_colmajor(n, n, torch.float64, device)
    Pc = P if P is not None else (empty_colmajor(m, n, dt, device) if return_p else None)
    info = torch.zeros(1, dtype=torch.int32, device=device)
    return dt, Zc, Qc, R, Pc, info, m, n


def qr_csr(row_ptr, col_idx, vals, Z, variant="ha", precision="fp64", reorth=False,
           return_p=False, Q=None, P=None, work=None, stream=None, device=None,
           panel=0, cgs=False, first=0, R=None) -> QRResult:
    """A-orthonormalise the columns of Z (device tensors; A in CSR).
    panel: 0 for the column schedule, 4 for the panel schedule, 8 for the
    two-level panel schedule (panels of eight, each as two of four), 16 for
    the three-level one (panels of sixteen, each as two of eight; naive and
    HA only); reorth:
    False, True (second pass per column) or 2 (blocked second pass, panel=8
    only); cgs: classical
    instead of modified Gram-Schmidt; first > 0: columns before it are final
    in the Q, P and R passed in (successive orthogonalisation).  stream: a
    torch stream or raw hipStream_t to run on (default: torch's current
    stream); the results are ready once that stream has reached them."""
    torch = _torch()
    device = device or Z.device
    with _on_stream(stream, device, (row_ptr, col_idx, vals, Z, Q, P, work, R)) as s:
        dt, Zc, Qc, R, Pc, info, m, n = _prep(Z, precision, device, Q, P, return_p, R)
        device = Zc.device
        vals = vals.to(device=device, dtype=dt).contiguous()
        row_ptr = row_ptr.to(device=device, dtype=torch.int32).contiguous()
        col_idx = col_idx.to(device=device, dtype=torch.int32).contiguous()
        h = handle(device.index or 0)
        opts = Opts(int(reorth), int(panel), int(bool(cgs)), int(first))
        v, p = VARIANTS[variant], PRECISIONS[precision]
        wb = amgs_workspace_bytes(h, m, n, 0, v, p, int(Pc is not None), opts)
        work = _workspace(work, wb, device)
        st = amgs_qr_csr(h, m, int(vals.numel()), row_ptr.data_ptr(), col_idx.data_ptr(),
                         vals.data_ptr(), n, Zc.data_ptr(), max(Zc.stride(1), m), Qc.data_ptr(),
                         max(Qc.stride(1), m), R.data_ptr(), max(R.stride(1), n, 1),
                         Pc.data_ptr() if Pc is not None else None,
                         max(Pc.stride(1), m) if Pc is not None else 0, v, p, C.byref(opts),
                         work.data_ptr(), work.numel() * work.element_size(), info.data_ptr(), s)
    _check(st, "amgs_qr_csr")
    return QRResult(Qc, R, Pc, info, amgs_get_stats(h))


def qr_dense(A, Z, variant="ha", precision="fp64", reorth=False, return_p=False, Q=None,
             P=None, work=None, stream=None, device=None, panel=0, cgs=False, first=0,
             R=None) -> QRResult:
    """A-orthonormalise the columns of Z (device tensors; A dense symmetric).
    panel: 0 for the column schedule, 4 for the panel schedule, 8 for the
    two-level panel schedule (panels of eight, each as two of four), 16 for
    the three-level one (panels of sixteen, each as two of eight; naive and
    HA only); reorth:
    False, True (second pass per column) or 2 (blocked second pass, panel=8
    only); cgs: classical
    instead of modified Gram-Schmidt; first > 0: columns before it are final
    in the Q, P and R passed in (successive orthogonalisation).  stream: as
    for qr_csr."""
    device = device or Z.device
    with _on_stream(stream, device, (A, Z, Q, P, work, R)) as s:
        dt, Zc, Qc, R, Pc, info, m, n = _prep(Z, precision, device, Q, P, return_p, R)
        device = Zc.device
        Ac = colmajor(A.to(device), dt)
        h = handle(device.index or 0)
        opts = Opts(int(reorth), int(panel), int(bool(cgs)), int(first))
        v, p = VARIANTS[variant], PRECISIONS[precision]
        wb = amgs_workspace_bytes(h, m, n, 1, v, p, int(Pc is not None), opts)
        work = _workspace(work, wb, device)
        st = amgs_qr_dense(h, m, Ac.data_ptr(), max(Ac.stride(1), m), n, Zc.data_ptr(),
                           max(Zc.stride(1), m), Qc.data_ptr(), max(Qc.stride(1), m),
                           R.data_ptr(), max(R.stride(1), n, 1),
                           Pc.data_ptr() if Pc is not None else None,
                           max(Pc.stride(1), m) if Pc is not None else 0, v, p, C.byref(opts),
                           work.data_ptr(), work.numel() * work.element_size(), info.data_ptr(),
                           s)
    _check(st, "amgs_qr_dense")
    return QRResult(Qc, R, Pc, info, amgs_get_stats(h))


def csr_check(row_ptr, col_idx, m: int) -> bool:
    torch = _torch()
    flag = torch.ones(1, dtype=torch.int32, device=row_ptr.device)
    h = handle(row_ptr.device.index or 0)
    s = torch.cuda.current_stream(row_ptr.device).cuda_stream
    _check(amgs_csr_check(h, m, int(col_idx.numel()), row_ptr.data_ptr(), col_idx.data_ptr(),
                          flag.data_ptr(), s), "amgs_csr_check")
    return int(flag.item()) == 0


# ------------------------------------------------------------------ batched
def amgs_batch_plan_create(h, batch, m_arr, n_arr, variant, precision, opts, autotune) -> int:
    plan = _vp()
    M = (_i64 * max(batch, 1))(*m_arr)
    N = (_i64 * max(batch, 1))(*n_arr)
    _check(load().amgs_batch_plan_create(h, batch, M, N, variant, precision,
                                         C.byref(opts) if opts is not None else None,
                                         autotune, C.byref(plan)), "amgs_batch_plan_create")
    return plan.value


def amgs_batch_plan_destroy(plan) -> int:
    return load().amgs_batch_plan_destroy(plan)


def amgs_batch_workspace_bytes(plan) -> int:
    return int(load().amgs_batch_workspace_bytes(plan))


def amgs_qr_batched(plan, desc_ptr, work_ptr, work_bytes, info_ptr, stream) -> int:
    return load().amgs_qr_batched(plan, desc_ptr, work_ptr, work_bytes, info_ptr, stream)


def amgs_batch_plan_tiles(plan):
    out = (_i32 * 16)()
    k = load().amgs_batch_plan_tiles(plan, out, 16)
    return [out[i] for i in range(k)]


class BatchPlan:
    """A plan for one list of instance shapes (see amgs_batch_plan_create)."""

    def __init__(self, ms, ns, variant="ha", precision="fp64", reorth=False, autotune=False,
                 device=0):
        self.h = handle(device)
        self.batch = len(ms)
        self.ms, self.ns = [int(x) for x in ms], [int(x) for x in ns]
        self.variant, self.precision, self.reorth = variant, precision, bool(reorth)
        self.opts = Opts(int(bool(reorth)), 0, 0, 0)
        self.plan = amgs_batch_plan_create(self.h, self.batch, list(ms), list(ns),
                                           VARIANTS[variant], PRECISIONS[precision], self.opts,
                                           int(bool(autotune)))

    def workspace_bytes(self) -> int:
        return amgs_batch_workspace_bytes(self.plan)

    def tiles(self):
        return amgs_batch_plan_tiles(self.plan)

    def run(self, desc, work, info, stream=None):
        """One pass over the plan's instances on `stream` (as for qr_csr)."""
        with _on_stream(stream, desc.device, (desc, work, info)) as s:
            _check(amgs_qr_batched(self.plan, desc.data_ptr(), work.data_ptr() if work is not None
                                   else None, work.numel() * work.element_size()
                                   if work is not None else 0,
                                   info.data_ptr(), s), "amgs_qr_batched")

    def __del__(self):
        try:
            if getattr(self, "plan", None):
                amgs_batch_plan_destroy(self.plan)
        except Exception:
            pass


def pack_descriptors(items, device):
    """items: list of dicts with device tensors row_ptr, col_idx, vals, Z, Q, R
    (Z, Q column-major m x n; R column-major n x n float64).  Returns a device
    uint8 tensor holding the amgs_batch_desc_t array."""
    torch = _torch()
    arr = (BatchDesc * max(len(items), 1))()
    for k, it in enumerate(items):
        Z, Q, R = it["Z"], it["Q"], it["R"]
        m, n = Z.shape
        arr[k] = BatchDesc(m, n, int(it["vals"].numel()), it["row_ptr"].data_ptr(),
                           it["col_idx"].data_ptr(), it["vals"].data_ptr(), Z.data_ptr(),
                           max(Z.stride(1), m), Q.data_ptr(), max(Q.stride(1), m), R.data_ptr(),
                           max(R.stride(1), n))
    raw = bytes(arr)[: C.sizeof(BatchDesc) * len(items)]
    host = torch.frombuffer(bytearray(raw), dtype=torch.uint8)
    return host.to(device)


def qr_batched(instances, variant="ha", precision="fp64", reorth=False, autotune=False,
               plan=None, stream=None):
    """instances: list of (row_ptr, col_idx, vals, Z) device tensors (CSR A, Z
    m x n).  Returns (Qs, Rs, info, plan, keep), keep holding the operands the
    launch uses.  stream: as for qr_csr; the descriptor copy, the outputs and
    the workspace are made on that stream."""
    torch = _torch()
    dt = torch.float64 if precision == "fp64" else torch.float32
    dev = instances[0][3].device
    ms = [int(Z.shape[0]) if Z.dim() == 2 else int(Z.numel()) for _, _, _, Z in instances]
    ns = [int(Z.shape[1]) if Z.dim() == 2 else 1 for _, _, _, Z in instances]
    if plan is None:
        plan = BatchPlan(ms, ns, variant, precision, reorth, autotune, dev.index or 0)
    elif (plan.ms, plan.ns) != (ms, ns) or (plan.variant, plan.precision, plan.reorth) != \
            (variant, precision, bool(reorth)):
        # the plan's workspace offsets are laid out for its own sizes
        raise ValueError("plan was created for other instance sizes or options")
    caller = [t for inst in instances for t in inst]
    with _on_stream(stream, dev, caller) as s:
        items, Qs, Rs = [], [], []
        for rp, ci, va, Z in instances:
            Zc = colmajor(Z, dt)
            m, n = Zc.shape
            Q = empty_colmajor(m, n, dt, dev)
            R = empty_colmajor(n, n, torch.float64, dev)
            items.append(dict(row_ptr=rp.to(torch.int32).contiguous(),
                              col_idx=ci.to(torch.int32).contiguous(),
                              vals=va.to(dt).contiguous(), Z=Zc, Q=Q, R=R))
            Qs.append(Q)
            Rs.append(R)
        desc = pack_descriptors(items, dev)
        work = torch.empty(max(plan.workspace_bytes(), 1), dtype=torch.uint8, device=dev)
        info = torch.full((len(items),), -7, dtype=torch.int32, device=dev)
        _check(amgs_qr_batched(plan.plan, desc.data_ptr(), work.data_ptr(),
                               work.numel() * work.element_size(), info.data_ptr(), s),
               "amgs_qr_batched")
    # keep the operands alive with the outputs
    return Qs, Rs, info, plan, (items, desc, work)
