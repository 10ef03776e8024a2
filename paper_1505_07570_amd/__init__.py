"""Python binding of librmm (randomized sketching on MI355X / gfx950).

Argument marshalling only: every operation runs in the HIP kernels of
``librmm.so``; PyTorch provides device memory and the current stream.  The
binding fails loudly when the library has not been built.

Matrices are torch tensors on the GPU in column-major layout
(``stride(0) == 1``), e.g. ``torch.empty(n, m, device="cuda").t()``; use
:func:`colmajor` to convert.
"""

from __future__ import annotations

import ctypes
import math
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librmm.so")

GAUSSIAN, SRHT, COUNTSKETCH = 0, 1, 2
KINDS = {"gaussian": GAUSSIAN, "srht": SRHT, "countsketch": COUNTSKETCH}
PREC_NATIVE, PREC_BF16, PREC_FP8 = 0, 1, 2
F32, F64 = 0, 1

STATUS_RANK_DEFICIENT = 1
STATUS_QR_FALLBACK = 2
STATUS_NOT_CONVERGED = 4
ERR_UNSUPPORTED = -4
ERR_SCRATCH_LIMIT = -5
NOALLOC_SCRATCH_BYTES = 128 << 20

_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_vp = ctypes.c_void_p
_i32 = ctypes.c_int


class RmmError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {_strerror(code)} ({code})")
        self.code = code


_lib = None


def lib():
    """The loaded librmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_1505_07570_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "rmm_create": [ctypes.POINTER(_vp), _i32],
            "rmm_destroy": [_vp],
            "rmm_set_stream": [_vp, _vp],
            "rmm_set_workspace": [_vp, _vp, ctypes.c_size_t],
            "rmm_device_cus": [_vp, ctypes.POINTER(_i32)],
            "rmm_set_autotune": [_vp, _i32],
            "rmm_set_kernel_timing": [_vp, _i32],
            "rmm_kernel_time": [_vp, ctypes.POINTER(ctypes.c_float)],
            "rmm_stream_read": [_vp, _vp, _i64, _vp],
            "rmm_autotune_count": [_vp, ctypes.POINTER(_i64)],
            "rmm_autotune_save": [_vp, ctypes.c_char_p],
            "rmm_autotune_load": [_vp, ctypes.c_char_p],
            "rmm_sketch_workspace": [_vp, _i32, _i32, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_sketch": [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _u64, _vp, _i64],
            "rmm_sketch_composite_workspace": [_vp, _i32, _i32, _i64, _i64, _i64, _i64,
                                               ctypes.POINTER(ctypes.c_size_t)],
            "rmm_sketch_composite": [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _i64, _u64,
                                     _vp, _i64],
            "rmm_rsvd_workspace": [_vp, _i32, _i32, _i64, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_rsvd_lanczos_workspace": [_vp, _i32, _i64, _i64, _i64, _i64, _i64,
                                           ctypes.POINTER(ctypes.c_size_t)],
            "rmm_rsvd_lanczos": [_vp, _i32, _i64, _i64, _vp, _i64, _i64, _i64, _i64, _u64, _vp, _i64,
                                 _vp, _vp, _i64, _vp],
            "rmm_rsvd_faster_workspace": [_vp, _i32, _i32, _i64, _i64, _i64, _i64, _i64, _i64,
                                          ctypes.POINTER(ctypes.c_size_t)],
            "rmm_rsvd_faster": [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _i64, _i64, _i64, _i64, _u64,
                                _vp, _i64, _vp, _vp, _i64, _vp],
            "rmm_rsvd": [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _i64, _i64, _i64, _u64,
                         _vp, _i64, _vp, _vp, _i64, _vp],
            "rmm_lsr_workspace": [_vp, _i32, _i32, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_sketched_lsr": [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _u64, _vp, _vp, _vp],
            "rmm_spsd_faster_workspace": [_vp, _i32, _i64, _i64, _i64, _i64,
                                          ctypes.POINTER(ctypes.c_size_t)],
            "rmm_spsd_faster": [_vp, _i32, _i64, _i64, _vp, _i64, ctypes.c_double, _i64, _i64, _u64,
                                _vp, _vp, _vp, _vp, _i64, _vp, _vp],
            "rmm_cur_faster_workspace": [_vp, _i32, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _i32,
                                         ctypes.POINTER(ctypes.c_size_t)],
            "rmm_cur_faster": [_vp, _i32, _i64, _i64, _i64, _vp, _i64, _vp, _i64, ctypes.c_double,
                               _i64, _i64, _i64, _i64, _i32, _u64, _vp, _vp, _vp, _vp, _vp, _vp, _i64,
                               _vp, _i64, _vp, _i64, _vp],
            "rmm_leverage_sample_workspace": [_vp, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_leverage_sample": [_vp, _i64, _vp, _i64, _i32, _u64, _vp],
            "rmm_sketched_lsr_noalloc": [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _u64, _vp,
                                         _vp, _vp],
            "rmm_precise_lsr_workspace": [_vp, _i32, _i32, _i64, _i64, _i64,
                                          ctypes.POINTER(ctypes.c_size_t)],
            "rmm_precise_lsr": [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _u64, _i64, _vp,
                                _vp, _vp],
            "rmm_plain_lsr_workspace": [_vp, _i32, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_plain_lsr": [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp],
            "rmm_lsr_solve_workspace": [_vp, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_lsr_solve": [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _vp],
            "rmm_residual_workspace": [_vp, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_residual": [_vp, _i32, _i64, _i64, _vp, _i64, _vp, _vp, _vp],
            "rmm_mixed_product_workspace": [_vp, _i32, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_mixed_product": [_vp, _i32, _i32, _i64, _i64, _vp, _i64, _vp, _i64, _i64, _vp, _i64],
            "rmm_nystrom_workspace": [_vp, _i64, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_nystrom": [_vp, _i64, _i64, _vp, _i64, ctypes.c_double, _i64, _i64, _u64, _vp, _vp,
                            _i64, _vp, _i64, _vp, _vp],
            "rmm_nystrom_gaussian_workspace": [_vp, _i64, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_nystrom_gaussian": [_vp, _i64, _i64, _vp, _i64, ctypes.c_double, _i64, _i64, _u64, _vp,
                                     _i64, _vp, _i64, _vp, _vp],
            "rmm_sketch_batch_workspace": [_vp, _i32, _i32, _i64, _vp, ctypes.POINTER(ctypes.c_size_t)],
            "rmm_sketch_batch": [_vp, _i32, _i32, _i64, _vp],
            "rmm_sched_create": [ctypes.c_size_t, ctypes.POINTER(_vp)],
            "rmm_sched_destroy": [_vp],
            "rmm_sched_submit": [_vp, _i64, ctypes.c_size_t],
            "rmm_sched_admit": [_vp, _i64, _vp, ctypes.POINTER(_i64)],
            "rmm_sched_complete": [_vp, _i64],
            "rmm_sched_stats": [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_i64),
                                ctypes.POINTER(_i64)],
            "rmm_sketch_hashes": [_vp, _i64, _i64, _u64, _vp],
            "rmm_sketch_signs": [_vp, _i32, _i64, _u64, _vp],
            "rmm_srht_indices": [_vp, _i64, _i64, _u64, _vp],
            "rmm_gaussian": [_vp, _i32, _i32, _i64, _i64, _u64, _vp, _i64],
        }
        for name, args in sig.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = _i32
        L.rmm_strerror.argtypes = [_i32]
        L.rmm_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().rmm_strerror(code).decode()
    except Exception:  # pragma: no cover - library missing
        return "error"


def _check(code: int, what: str):
    if code != 0:
        raise RmmError(code, what)


def _dt(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _kind(kind) -> int:
    if isinstance(kind, str):
        return KINDS[kind.lower()]
    return int(kind)


def colmajor(x: torch.Tensor) -> torch.Tensor:
    """Column-major copy (or the tensor itself if it already is one)."""
    if x.dim() == 1:
        return x.contiguous()
    if x.stride(0) == 1 and x.stride(1) >= max(1, x.shape[0]):
        return x
    return x.t().contiguous().t()


def _ld(x: torch.Tensor) -> int:
    if x.dim() == 1:
        return max(1, x.shape[0])
    if x.stride(0) != 1 and x.shape[0] > 1:
        raise ValueError("matrix must be column-major (stride(0) == 1)")
    return max(1, x.stride(1), x.shape[0])


def _ptr(x):
    return None if x is None else ctypes.c_void_p(x.data_ptr())


def _bptr(b, out):
    """Pointer of the optional extra column.  NULL means "no column", so an
    empty column (zero rows, no storage) is passed as a non-null pointer that
    is never read (the output's)."""
    if b is None:
        return None
    return ctypes.c_void_p(b.data_ptr() if b.numel() > 0 else out.data_ptr())


class SketchDesc(ctypes.Structure):
    """rmm_sketch_desc of the C ABI."""
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("A", ctypes.c_void_p),
                ("lda", ctypes.c_int64), ("b", ctypes.c_void_p), ("s", ctypes.c_int64),
                ("seed", ctypes.c_uint64), ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64)]


class Scheduler:
    """First-come-first-served admission under a device-memory budget
    (host-only; the rmm_sched_* calls of the C ABI)."""

    def __init__(self, budget_bytes: int):
        s = ctypes.c_void_p()
        _check(lib().rmm_sched_create(ctypes.c_size_t(budget_bytes), ctypes.byref(s)), "rmm_sched_create")
        self._s = s

    def __del__(self):
        try:
            if self._s:
                lib().rmm_sched_destroy(self._s)
        except Exception:
            pass

    def submit(self, rid: int, nbytes: int):
        _check(lib().rmm_sched_submit(self._s, rid, ctypes.c_size_t(nbytes)), "rmm_sched_submit")

    def admit(self, max_ids: int = 1 << 16):
        ids = (ctypes.c_int64 * max(1, max_ids))()
        n = ctypes.c_int64()
        _check(lib().rmm_sched_admit(self._s, max_ids, ids, ctypes.byref(n)), "rmm_sched_admit")
        return list(ids[:n.value])

    def complete(self, rid: int):
        _check(lib().rmm_sched_complete(self._s, rid), "rmm_sched_complete")

    def stats(self):
        u = ctypes.c_size_t()
        q = ctypes.c_int64()
        r = ctypes.c_int64()
        _check(lib().rmm_sched_stats(self._s, ctypes.byref(u), ctypes.byref(q), ctypes.byref(r)),
               "rmm_sched_stats")
        return {"in_use": u.value, "queued": q.value, "running": r.value}


class Handle:
    """A library handle bound to one device, its stream and a workspace."""

    def __init__(self, device=None):
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.device = device
        h = ctypes.c_void_p()
        _check(lib().rmm_create(ctypes.byref(h), device.index or 0), "rmm_create")
        self._h = h
        self._ws = None
        self._ws_streams = set()

    def __del__(self):
        try:
            if self._h:
                lib().rmm_destroy(self._h)
        except Exception:
            pass

    @property
    def cus(self) -> int:
        v = ctypes.c_int()
        _check(lib().rmm_device_cus(self._h, ctypes.byref(v)), "rmm_device_cus")
        return v.value

    def _prepare(self, nbytes: int):
        """Bind the current torch stream and a workspace of >= nbytes."""
        stream = torch.cuda.current_stream(self.device)
        _check(lib().rmm_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), "rmm_set_stream")
        if self._ws is not None and stream not in self._ws_streams:
            # work on another stream uses the workspace: the allocator must not
            # hand its memory out again before that work is done
            self._ws.record_stream(stream)
            self._ws_streams.add(stream)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self._ws_streams = {stream}
        _check(lib().rmm_set_workspace(self._h, _ptr(self._ws), self._ws.numel()),
               "rmm_set_workspace")

    def _bind_stream(self):
        """Bind the current torch stream only (no workspace)."""
        stream = torch.cuda.current_stream(self.device)
        _check(lib().rmm_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), "rmm_set_stream")

    def reserve(self, nbytes: int):
        self._prepare(nbytes)

    # ---- sketching -------------------------------------------------------
    def sketch_composite_workspace(self, dtype, kind2, m, ncols, s1, s) -> int:
        out = ctypes.c_size_t()
        dt = F32 if dtype == torch.float32 else F64
        _check(lib().rmm_sketch_composite_workspace(self._h, dt, _kind(kind2), m, ncols, s1, s,
                                                    ctypes.byref(out)), "rmm_sketch_composite_workspace")
        return out.value

    def sketch_composite(self, A: torch.Tensor, s1: int, s: int, kind2, seed: int,
                         b: torch.Tensor = None, out: torch.Tensor = None) -> torch.Tensor:
        """C = (S_cs S_2)^T [A | b] (s x n'): CountSketch to s1 rows, then kind2 to s."""
        A = colmajor(A)
        m, n = A.shape
        ncols = n + (1 if b is not None else 0)
        if out is None:
            out = torch.empty(ncols, s, dtype=A.dtype, device=A.device).t()
        ws = self.sketch_composite_workspace(A.dtype, kind2, m, ncols, s1, s)
        self._prepare(ws)
        _check(lib().rmm_sketch_composite(self._h, _dt(A), _kind(kind2), m, n, _ptr(A), _ld(A),
                                          _bptr(b, out), s1, s, seed, _ptr(out), _ld(out)),
               "rmm_sketch_composite")
        return out

    def sketch_workspace(self, dtype, kind, m, ncols, s) -> int:
        out = ctypes.c_size_t()
        dt = F32 if dtype == torch.float32 else F64
        _check(lib().rmm_sketch_workspace(self._h, dt, _kind(kind), m, ncols, s, ctypes.byref(out)),
               "rmm_sketch_workspace")
        return out.value

    def sketch(self, A: torch.Tensor, s: int, kind, seed: int, b: torch.Tensor = None,
               out: torch.Tensor = None) -> torch.Tensor:
        """C = S^T [A | b] (s x n'), column-major, same dtype as A."""
        A = colmajor(A)
        m, n = A.shape
        ncols = n + (1 if b is not None else 0)
        if out is None:
            out = torch.empty(ncols, s, dtype=A.dtype, device=A.device).t()
        ws = self.sketch_workspace(A.dtype, kind, m, ncols, s)
        self._prepare(ws)
        _check(lib().rmm_sketch(self._h, _dt(A), _kind(kind), m, n, _ptr(A), _ld(A), _bptr(b, out), s,
                                seed, _ptr(out), _ld(out)), "rmm_sketch")
        return out

    # ---- randomized SVD ----------------------------------------------------
    def rsvd(self, A: torch.Tensor, k: int, p: int, q: int, seed: int, prec: int = PREC_NATIVE):
        A = colmajor(A)
        m, n = A.shape
        dt = _dt(A)
        U = torch.empty(k, m, dtype=A.dtype, device=A.device).t()
        V = torch.empty(k, n, dtype=A.dtype, device=A.device).t()
        sig = torch.empty(k, dtype=A.dtype, device=A.device)
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_rsvd_workspace(self._h, dt, prec, m, n, k, p, ctypes.byref(ws)),
               "rmm_rsvd_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_rsvd(self._h, dt, prec, m, n, _ptr(A), _ld(A), k, p, q, seed, _ptr(U),
                              _ld(U), _ptr(sig), _ptr(V), _ld(V), _ptr(status)), "rmm_rsvd")
        return U, sig, V, status

    def rsvd_lanczos(self, A: torch.Tensor, k: int, s: int, q: int, seed: int):
        """Alg. 5.1 with q Krylov blocks of width s: (U, sigma, V, status)."""
        A = colmajor(A)
        m, n = A.shape
        dt = _dt(A)
        U = torch.empty(k, m, dtype=A.dtype, device=A.device).t()
        V = torch.empty(k, n, dtype=A.dtype, device=A.device).t()
        sig = torch.empty(k, dtype=A.dtype, device=A.device)
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_rsvd_lanczos_workspace(self._h, dt, m, n, k, s, q, ctypes.byref(ws)),
               "rmm_rsvd_lanczos_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_rsvd_lanczos(self._h, dt, m, n, _ptr(A), _ld(A), k, s, q, seed, _ptr(U),
                                      _ld(U), _ptr(sig), _ptr(V), _ld(V), _ptr(status)),
               "rmm_rsvd_lanczos")
        return U, sig, V, status

    def rsvd_faster(self, A: torch.Tensor, k: int, s: int, p_cs: int, p: int, seed: int,
                    kind2="srht"):
        """Alg. 5.3: (U, sigma, V, status); see rmm_rsvd_faster."""
        A = colmajor(A)
        m, n = A.shape
        dt = _dt(A)
        U = torch.empty(k, m, dtype=A.dtype, device=A.device).t()
        V = torch.empty(k, n, dtype=A.dtype, device=A.device).t()
        sig = torch.empty(k, dtype=A.dtype, device=A.device)
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_rsvd_faster_workspace(self._h, dt, _kind(kind2), m, n, k, s, p_cs, p,
                                               ctypes.byref(ws)), "rmm_rsvd_faster_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_rsvd_faster(self._h, dt, _kind(kind2), m, n, _ptr(A), _ld(A), k, s, p_cs, p,
                                     seed, _ptr(U), _ld(U), _ptr(sig), _ptr(V), _ld(V), _ptr(status)),
               "rmm_rsvd_faster")
        return U, sig, V, status

    # ---- autotuning of the dense products (rmm_set_autotune) -------------------
    def set_autotune(self, on: bool = True):
        _check(lib().rmm_set_autotune(self._h, 1 if on else 0), "rmm_set_autotune")

    def autotune_count(self) -> int:
        n = ctypes.c_int64()
        _check(lib().rmm_autotune_count(self._h, ctypes.byref(n)), "rmm_autotune_count")
        return n.value

    def autotune_save(self, path: str):
        _check(lib().rmm_autotune_save(self._h, path.encode()), "rmm_autotune_save")

    def autotune_load(self, path: str):
        _check(lib().rmm_autotune_load(self._h, path.encode()), "rmm_autotune_load")

    # ---- timing of the sketches' main kernels (rmm_set_kernel_timing) ------------
    def set_kernel_timing(self, on: bool = True):
        _check(lib().rmm_set_kernel_timing(self._h, 1 if on else 0), "rmm_set_kernel_timing")

    def stream_read(self, x: torch.Tensor, sink: torch.Tensor):
        """One streaming read of x (the HBM read reference); sink: >= 4096 float32."""
        assert x.is_cuda and x.is_contiguous() and sink.dtype == torch.float32 and sink.numel() >= 4096
        self._bind_stream()
        _check(lib().rmm_stream_read(self._h, _ptr(x), x.numel() * x.element_size(), _ptr(sink)),
               "rmm_stream_read")

    def kernel_time(self) -> float:
        """Milliseconds of the last timed sketch kernel (waits for it)."""
        ms = ctypes.c_float()
        _check(lib().rmm_kernel_time(self._h, ctypes.byref(ms)), "rmm_kernel_time")
        return float(ms.value)

    # ---- least squares -------------------------------------------------------
    def sketched_lsr(self, A: torch.Tensor, b: torch.Tensor, s: int, kind, seed: int,
                     residual: bool = True):
        A = colmajor(A)
        m, d = A.shape
        dt = _dt(A)
        x = torch.empty(d, dtype=torch.float64, device=A.device)
        res = torch.empty(1, dtype=torch.float64, device=A.device) if residual else None
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_lsr_workspace(self._h, dt, _kind(kind), m, d, s, ctypes.byref(ws)),
               "rmm_lsr_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_sketched_lsr(self._h, dt, _kind(kind), m, d, _ptr(A), _ld(A), _ptr(b), s,
                                      seed, _ptr(x), _ptr(res), _ptr(status)), "rmm_sketched_lsr")
        return x, res, status

    def sketched_lsr_noalloc(self, A: torch.Tensor, b: torch.Tensor, s: int, kind, seed: int,
                             residual: bool = True):
        """sketched_lsr with the library's static device scratch instead of the
        handle's workspace (the workspace is neither grown nor used)."""
        A = colmajor(A)
        m, d = A.shape
        dt = _dt(A)
        x = torch.empty(d, dtype=torch.float64, device=A.device)
        res = torch.empty(1, dtype=torch.float64, device=A.device) if residual else None
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
        self._bind_stream()
        _check(lib().rmm_sketched_lsr_noalloc(self._h, dt, _kind(kind), m, d, _ptr(A), _ld(A),
                                              _ptr(b), s, seed, _ptr(x), _ptr(res), _ptr(status)),
               "rmm_sketched_lsr_noalloc")
        return x, res, status

    def precise_lsr(self, A: torch.Tensor, b: torch.Tensor, s: int, kind, seed: int, iters: int,
                    residual: bool = True):
        """Alg. 4.1: sketch-and-solve start, then `iters` preconditioned CG steps."""
        A = colmajor(A)
        m, d = A.shape
        dt = _dt(A)
        x = torch.empty(d, dtype=torch.float64, device=A.device)
        res = torch.empty(1, dtype=torch.float64, device=A.device) if residual else None
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_precise_lsr_workspace(self._h, dt, _kind(kind), m, d, s, ctypes.byref(ws)),
               "rmm_precise_lsr_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_precise_lsr(self._h, dt, _kind(kind), m, d, _ptr(A), _ld(A), _ptr(b), s,
                                     seed, iters, _ptr(x), _ptr(res), _ptr(status)),
               "rmm_precise_lsr")
        return x, res, status

    def lsr_solve(self, Cs: torch.Tensor, d: int):
        """x = argmin ||Cs[:, :d] x - Cs[:, d]|| for a sketched system Cs."""
        s = Cs.shape[0]
        x = torch.empty(d, dtype=torch.float64, device=Cs.device)
        status = torch.zeros(1, dtype=torch.int32, device=Cs.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_lsr_solve_workspace(self._h, s, d, ctypes.byref(ws)), "rmm_lsr_solve_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_lsr_solve(self._h, _dt(Cs), s, d, _ptr(Cs), _ld(Cs), _ptr(x), _ptr(status)),
               "rmm_lsr_solve")
        return x, status

    def residual(self, A: torch.Tensor, b: torch.Tensor, x: torch.Tensor, out: torch.Tensor = None):
        """||A x - b||_2 in fp64 (x: fp64 device vector)."""
        A = colmajor(A)
        m, d = A.shape
        out = torch.empty(1, dtype=torch.float64, device=A.device) if out is None else out
        ws = ctypes.c_size_t()
        _check(lib().rmm_residual_workspace(self._h, m, ctypes.byref(ws)), "rmm_residual_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_residual(self._h, _dt(A), m, d, _ptr(A), _ld(A), _ptr(b), _ptr(x), _ptr(out)),
               "rmm_residual")
        return out

    def plain_lsr(self, A: torch.Tensor, b: torch.Tensor, residual: bool = True):
        A = colmajor(A)
        m, d = A.shape
        dt = _dt(A)
        x = torch.empty(d, dtype=torch.float64, device=A.device)
        res = torch.empty(1, dtype=torch.float64, device=A.device) if residual else None
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_plain_lsr_workspace(self._h, dt, m, d, ctypes.byref(ws)),
               "rmm_plain_lsr_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_plain_lsr(self._h, dt, m, d, _ptr(A), _ld(A), _ptr(b), _ptr(x), _ptr(res),
                                   _ptr(status)), "rmm_plain_lsr")
        return x, res, status

    def mixed_product(self, A: torch.Tensor, X: torch.Tensor, prec: int, mode: int) -> torch.Tensor:
        """Quantized A X (mode 0) or A^T X (mode 1), fp32 accumulation."""
        A = colmajor(A)
        X = colmajor(X)
        m, n = A.shape
        l = X.shape[1]
        rows = m if mode == 0 else n
        out = torch.empty(l, rows, dtype=torch.float32, device=A.device).t()
        ws = ctypes.c_size_t()
        _check(lib().rmm_mixed_product_workspace(self._h, prec, m, n, l, ctypes.byref(ws)),
               "rmm_mixed_product_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_mixed_product(self._h, prec, mode, m, n, _ptr(A), _ld(A), _ptr(X), _ld(X), l,
                                       _ptr(out), _ld(out)), "rmm_mixed_product")
        return out

    def sketch_batch_workspace(self, kind, shapes, dtype=torch.float32) -> int:
        """Workspace bytes of sketch_batch for problems of the given
        (m, n, with_b, s) shapes (the size query reads no operand: the
        descriptors carry placeholder addresses)."""
        descs = (SketchDesc * max(1, len(shapes)))()
        for i, (m, n, with_b, s) in enumerate(shapes):
            descs[i] = SketchDesc(m, n, 256, max(1, m), 256 if with_b else None, s, 0, 256, max(1, s))
        dt = F32 if dtype == torch.float32 else F64
        ws = ctypes.c_size_t()
        _check(lib().rmm_sketch_batch_workspace(self._h, dt, _kind(kind), len(shapes), descs,
                                                ctypes.byref(ws)), "rmm_sketch_batch_workspace")
        return ws.value

    def sketch_batch(self, kind, problems, dtype=torch.float32):
        """Sketches of several problems in one grouped call.

        problems: list of (A, b or None, s, seed); returns the list of C_i
        (s_i x n_i', column-major), each bitwise equal to sketch() alone."""
        descs = (SketchDesc * max(1, len(problems)))()
        outs, keep = [], []
        for i, (A, b, s, seed) in enumerate(problems):
            A = colmajor(A)
            keep.append(A)
            m, n = A.shape
            ncols = n + (1 if b is not None else 0)
            C = torch.empty(ncols, s, dtype=A.dtype, device=A.device).t()
            outs.append(C)
            bp = _bptr(b, C)
            descs[i] = SketchDesc(m, n, A.data_ptr(), _ld(A), None if bp is None else bp.value, s, seed,
                                  C.data_ptr(), _ld(C))
        dt = F32 if dtype == torch.float32 else F64
        ws = ctypes.c_size_t()
        _check(lib().rmm_sketch_batch_workspace(self._h, dt, _kind(kind), len(problems), descs,
                                                ctypes.byref(ws)), "rmm_sketch_batch_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_sketch_batch(self._h, dt, _kind(kind), len(problems), descs), "rmm_sketch_batch")
        return outs

    # ---- Nystrom --------------------------------------------------------------
    def nystrom(self, X: torch.Tensor, sigma: float, c: int, seed: int, k: int = None):
        """RBF-kernel Nystrom factor of the rows of X (n x d, fp32, row-major).

        Returns (L (n x k), idx (c), C (n x c), evals (c), status)."""
        if X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
            X = X.to(torch.float32).contiguous()
        n, d = X.shape
        k = int(math.ceil(0.8 * c)) if k is None else int(k)
        idx = torch.empty(c, dtype=torch.int64, device=X.device)
        C = torch.empty(c, n, dtype=torch.float32, device=X.device).t()
        L = torch.empty(k, n, dtype=torch.float32, device=X.device).t()
        evals = torch.empty(c, dtype=torch.float64, device=X.device)
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_nystrom_workspace(self._h, n, d, c, k, ctypes.byref(ws)), "rmm_nystrom_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_nystrom(self._h, n, d, _ptr(X), X.stride(0), float(sigma), c, k, seed, _ptr(idx),
                                 _ptr(C), _ld(C), _ptr(L), _ld(L), _ptr(evals), _ptr(status)),
               "rmm_nystrom")
        return L, idx, C, evals, status

    def spsd_faster(self, X: torch.Tensor, sigma: float, s: int, p: int, seed: int):
        """Alg. 6.1 on the RBF kernel of the rows of X (n x d, fp32 or fp64,
        row-major).  Returns (Qc (n x s fp64), Z (s x s fp64), S (s), P
        (sorted, P[:np]), status); K ~ Qc Z Qc^T."""
        if X.dtype not in (torch.float32, torch.float64) or X.dim() != 2 or X.stride(1) != 1:
            X = X.to(torch.float32).contiguous()
        n, d = X.shape
        dt = _dt(X)
        S = torch.empty(s, dtype=torch.int64, device=X.device)
        P = torch.empty(p + s, dtype=torch.int64, device=X.device)
        npd = torch.empty(1, dtype=torch.int64, device=X.device)
        Qc = torch.empty(s, n, dtype=torch.float64, device=X.device).t()
        Z = torch.empty(s, s, dtype=torch.float64, device=X.device).t()
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_spsd_faster_workspace(self._h, dt, n, d, s, p, ctypes.byref(ws)),
               "rmm_spsd_faster_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_spsd_faster(self._h, dt, n, d, _ptr(X), X.stride(0), float(sigma), s, p, seed,
                                     _ptr(S), _ptr(P), _ptr(npd), _ptr(Qc), _ld(Qc), _ptr(Z),
                                     _ptr(status)), "rmm_spsd_faster")
        return Qc, Z, S, P[:int(npd.item())], status

    def cur_faster(self, Xtest: torch.Tensor, Xtrain: torch.Tensor, sigma: float, c: int, r: int,
                   pc: int, pr: int, seed: int, mode: str = "uniform"):
        """Faster CUR of the RBF kernel K(Xtest, Xtrain) (Sec. 6.6.3).  Returns
        (C (m x c), U (c x r fp64), R (r x n), SC, SR, PC, PR, status)."""
        dt0 = Xtest.dtype if Xtest.dtype in (torch.float32, torch.float64) else torch.float32
        Xtest = Xtest.to(dt0).contiguous()
        Xtrain = Xtrain.to(dt0).contiguous()
        m, d = Xtest.shape
        n = Xtrain.shape[0]
        dt = _dt(Xtest)
        md = {"uniform": 0, "leverage": 1}[mode]
        dev = Xtest.device
        SC = torch.empty(c, dtype=torch.int64, device=dev)
        SR = torch.empty(r, dtype=torch.int64, device=dev)
        PC = torch.empty(pc + r, dtype=torch.int64, device=dev)
        PR = torch.empty(pr + c, dtype=torch.int64, device=dev)
        lens = torch.empty(2, dtype=torch.int64, device=dev)
        C = torch.empty(c, m, dtype=dt0, device=dev).t()
        U = torch.empty(r, c, dtype=torch.float64, device=dev).t()
        Rt = torch.empty(r, n, dtype=dt0, device=dev).t()
        status = torch.zeros(1, dtype=torch.int32, device=dev)
        ws = ctypes.c_size_t()
        _check(lib().rmm_cur_faster_workspace(self._h, dt, m, n, d, c, r, pc, pr, md, ctypes.byref(ws)),
               "rmm_cur_faster_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_cur_faster(self._h, dt, m, n, d, _ptr(Xtest), Xtest.stride(0), _ptr(Xtrain),
                                    Xtrain.stride(0), float(sigma), c, r, pc, pr, md, seed, _ptr(SC),
                                    _ptr(SR), _ptr(PC), _ptr(PR), _ptr(lens), _ptr(C), _ld(C), _ptr(U),
                                    _ld(U), _ptr(Rt), _ld(Rt), _ptr(status)), "rmm_cur_faster")
        ln = lens.tolist()
        return C, U, Rt.t(), SC, SR, PC[:ln[0]], PR[:ln[1]], status

    def leverage_sample(self, q: torch.Tensor, p: int, tag: int, seed: int):
        """p indices drawn with probability ~ q (the sampler of Alg. 6.1)."""
        q = q.to(torch.float64).contiguous()
        out = torch.empty(p, dtype=torch.int64, device=q.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_leverage_sample_workspace(self._h, q.numel(), ctypes.byref(ws)),
               "rmm_leverage_sample_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_leverage_sample(self._h, q.numel(), _ptr(q), p, tag, seed, _ptr(out)),
               "rmm_leverage_sample")
        return out

    def nystrom_gaussian(self, X: torch.Tensor, sigma: float, c: int, seed: int, k: int = None):
        """Gaussian-projection Nystrom: returns (L (n x k), C = K Omega (n x c), evals, status)."""
        if X.dtype != torch.float32 or X.dim() != 2 or X.stride(1) != 1:
            X = X.to(torch.float32).contiguous()
        n, d = X.shape
        k = int(math.ceil(0.8 * c)) if k is None else int(k)
        C = torch.empty(c, n, dtype=torch.float32, device=X.device).t()
        L = torch.empty(k, n, dtype=torch.float32, device=X.device).t()
        evals = torch.empty(c, dtype=torch.float64, device=X.device)
        status = torch.zeros(1, dtype=torch.int32, device=X.device)
        ws = ctypes.c_size_t()
        _check(lib().rmm_nystrom_gaussian_workspace(self._h, n, d, c, k, ctypes.byref(ws)),
               "rmm_nystrom_gaussian_workspace")
        self._prepare(ws.value)
        _check(lib().rmm_nystrom_gaussian(self._h, n, d, _ptr(X), X.stride(0), float(sigma), c, k, seed,
                                          _ptr(C), _ld(C), _ptr(L), _ld(L), _ptr(evals), _ptr(status)),
               "rmm_nystrom_gaussian")
        return L, C, evals, status

    # ---- random quantities ---------------------------------------------------
    def sketch_hashes(self, m: int, s: int, seed: int) -> torch.Tensor:
        out = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)[:m]
        self._prepare(0)
        _check(lib().rmm_sketch_hashes(self._h, m, s, seed, _ptr(out)), "rmm_sketch_hashes")
        return out

    def sketch_signs(self, kind, m: int, seed: int) -> torch.Tensor:
        out = torch.empty(max(m, 1), dtype=torch.int8, device=self.device)[:m]
        self._prepare(0)
        _check(lib().rmm_sketch_signs(self._h, _kind(kind), m, seed, _ptr(out)), "rmm_sketch_signs")
        return out

    def srht_indices(self, m: int, s: int, seed: int) -> torch.Tensor:
        out = torch.empty(s, dtype=torch.int64, device=self.device)
        self._prepare(0)
        _check(lib().rmm_srht_indices(self._h, m, s, seed, _ptr(out)), "rmm_srht_indices")
        return out

    def gaussian(self, rows: int, cols: int, seed: int, stream: int = 0,
                 dtype=torch.float64) -> torch.Tensor:
        out = torch.empty(max(cols, 1), max(rows, 1), dtype=dtype, device=self.device).t()[:rows, :cols]
        self._prepare(0)
        _check(lib().rmm_gaussian(self._h, F32 if dtype == torch.float32 else F64, stream, rows,
                                  cols, seed, _ptr(out), max(1, rows)), "rmm_gaussian")
        return out


_default = {}


def handle(device=None) -> Handle:
    """Per-device default handle."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    key = dev.index or 0
    if key not in _default:
        _default[key] = Handle(dev)
    return _default[key]


def sketch(A, s, kind, seed, b=None):
    return handle(A.device).sketch(A, s, kind, seed, b)


def rsvd(A, k, p, q, seed, prec=PREC_NATIVE):
    return handle(A.device).rsvd(A, k, p, q, seed, prec)


def sketched_lsr(A, b, s, kind, seed, residual=True):
    return handle(A.device).sketched_lsr(A, b, s, kind, seed, residual)


def precise_lsr(A, b, s, kind, seed, iters, residual=True):
    return handle(A.device).precise_lsr(A, b, s, kind, seed, iters, residual)


def plain_lsr(A, b, residual=True):
    return handle(A.device).plain_lsr(A, b, residual)
