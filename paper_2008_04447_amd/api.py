"""Thin Python binding of the C ABI (argument marshalling only).

Matrices are torch tensors on a HIP device in column-major layout: a (m, n)
tensor with strides (1, ld).  ``colmajor`` / ``empty_colmajor`` produce them.
PyTorch supplies device memory and the stream; every computation runs in
librqrcp.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import RQ_FP64, RQ_MIXED_BF16, RQError

_DT = {torch.float64: RQ_FP64, torch.float32: RQ_MIXED_BF16}


def empty_colmajor(m, n, dtype=torch.float64, device="cuda"):
    return torch.empty((max(n, 1), max(m, 1)), dtype=dtype, device=device).t()[:m, :n]


def colmajor(a, dtype=torch.float64, device="cuda"):
    """Column-major device copy of a 2-D array (numpy or torch)."""
    src = torch.as_tensor(a, dtype=dtype)
    m, n = src.shape
    out = empty_colmajor(m, n, dtype, device)
    out.copy_(src)
    return out


def ld(t):
    """Leading dimension of a column-major 2-D tensor (checks the layout)."""
    m, n = t.shape
    if n > 1 and m > 1 and t.stride(0) != 1:
        raise ValueError("tensor is not column-major (stride(0) must be 1)")
    return max(1, t.stride(1) if n > 1 else m)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check(fn, rc, h=None):
    if rc != 0:
        detail = ""
        if h is not None and h.ptr:
            detail = (_lib.load().rq_last_error(h.ptr) or b"").decode(errors="replace")
        raise RQError(fn, rc, detail)


class Handle:
    """Library handle bound to a device and a stream (default: current stream)."""

    def __init__(self, device=0, stream=None):
        lib = _lib.load()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        idx = self.device.index or 0
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ptr = ctypes.c_void_p()
        _check("rq_create", lib.rq_create(ctypes.byref(self.ptr), idx,
                                          ctypes.c_void_p(self.stream.cuda_stream)))

    def set_stream(self, stream):
        self.stream = stream
        _check("rq_set_stream", _lib.load().rq_set_stream(self.ptr, ctypes.c_void_p(stream.cuda_stream)))

    def sync(self):
        """Wait for the stream; raise RQError(RQ_E_DEVICE) on a device-side error."""
        err = ctypes.c_int64(0)
        rc = _lib.load().rq_sync_status(self.ptr, ctypes.byref(err))
        if rc != 0:
            raise RQError("rq_sync_status", rc, f"device_error bits = {err.value}")
        return 0

    def workspace_query(self, op, m, n, k, b, p, prec=RQ_FP64):
        """Workspace bytes the entry point ``op`` (an RQ_OP_* code) needs."""
        out = ctypes.c_size_t(0)
        _check("rq_workspace_query", _lib.load().rq_workspace_query(
            self.ptr, int(op), int(prec), m, n, k, b, p, ctypes.byref(out)))
        return out.value

    def workspace_reserve(self, nbytes):
        _check("rq_workspace_reserve", _lib.load().rq_workspace_reserve(self.ptr, int(nbytes)), self)

    def workspace_size(self):
        out = ctypes.c_size_t(0)
        _check("rq_workspace_size", _lib.load().rq_workspace_size(self.ptr, ctypes.byref(out)))
        return out.value

    def close(self):
        if self.ptr:
            _lib.load().rq_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_handle(device=None):
    dev = torch.cuda.current_device() if device is None else device
    stream = torch.cuda.current_stream(dev)
    h = _default.get(dev)
    if h is None:
        h = Handle(dev, stream)
        _default[dev] = h
    elif h.stream.cuda_stream != stream.cuda_stream:
        h.set_stream(stream)
    return h


def rqrcp_factor(A, Omega, b, p, k=None, handle=None):
    """RQRCP (Algorithm 4) in place on the column-major float64 tensor A.

    Returns (jpvt, tau, T, info) as device tensors; A holds R and the
    reflectors, info (one int64) is 0 or the 1-based column at which R11 was
    numerically singular and fresh samples replaced the sample update.
    """
    h = handle or default_handle(A.device.index)
    m, n = A.shape
    k = min(m, n) if k is None else int(k)
    dev = A.device
    jpvt = torch.empty(max(n, 1), dtype=torch.int64, device=dev)[:n]
    tau = torch.empty(max(k, 1), dtype=torch.float64, device=dev)[:k]
    T = empty_colmajor(b, max(k, 1), torch.float64, dev)
    info = torch.zeros(1, dtype=torch.int64, device=dev)
    rc = _lib.load().rqrcp_factor(h.ptr, m, n, k, b, p, _ptr(A), ld(A), _ptr(Omega),
                                  ld(Omega), _ptr(jpvt), _ptr(tau), _ptr(T), ld(T), _ptr(info))
    _check("rqrcp_factor", rc, h)
    return jpvt, tau, T, info


def rsrqrcp_factor(A, Omegas, b, p, k=None, handle=None):
    """RQRCP with repeated sampling (Section 3.4) in place on A.

    Omegas is a float64 device tensor of ceil(k / b) column-major ell x m
    slices (shape (nblk, m, ell) with unit stride along ell, i.e. slice J is
    Omegas[J].T); block J uses the first m - J b columns of slice J.
    Returns (jpvt, tau, T) like rqrcp_factor."""
    h = handle or default_handle(A.device.index)
    m, n = A.shape
    k = min(m, n) if k is None else int(k)
    ell = b + p
    nblk = (k + b - 1) // b
    if Omegas.dim() != 3 or Omegas.shape[0] < nblk or Omegas.shape[1] != m or \
            Omegas.shape[2] != ell or Omegas.stride(2) != 1 or Omegas.stride(1) < ell:
        raise ValueError("Omegas must be (nblk, m, ell) with unit stride along ell")
    dev = A.device
    jpvt = torch.empty(max(n, 1), dtype=torch.int64, device=dev)[:n]
    tau = torch.empty(max(k, 1), dtype=torch.float64, device=dev)[:k]
    T = empty_colmajor(b, max(k, 1), torch.float64, dev)
    rc = _lib.load().rsrqrcp_factor(h.ptr, m, n, k, b, p, _ptr(A), ld(A), _ptr(Omegas),
                                    Omegas.stride(1), Omegas.stride(0), _ptr(jpvt), _ptr(tau),
                                    _ptr(T), ld(T))
    _check("rsrqrcp_factor", rc, h)
    return jpvt, tau, T


def qrcp_factor(A, k=None, nb=32, handle=None):
    """Plain QRCP (Algorithm 2) in place on A; returns (jpvt, tau)."""
    h = handle or default_handle(A.device.index)
    m, n = A.shape
    k = min(m, n) if k is None else int(k)
    dev = A.device
    jpvt = torch.empty(max(n, 1), dtype=torch.int64, device=dev)[:n]
    tau = torch.empty(max(k, 1), dtype=torch.float64, device=dev)[:k]
    rc = _lib.load().qrcp_factor(h.ptr, m, n, k, nb, _ptr(A), ld(A), _ptr(jpvt), _ptr(tau))
    _check("qrcp_factor", rc, h)
    return jpvt, tau


def trqrcp_truncate(A, Omega, b, p, k, handle=None):
    """TRQRCP (Algorithm 5).  A float64 (FP64 path) or float32 (mixed BF16 path).

    Returns (jpvt, Y, T, R)."""
    h = handle or default_handle(A.device.index)
    m, n = A.shape
    dev = A.device
    prec = _DT[A.dtype]
    jpvt = torch.empty(max(n, 1), dtype=torch.int64, device=dev)[:n]
    Y = empty_colmajor(m, k, torch.float64, dev)
    T = empty_colmajor(k, k, torch.float64, dev)
    R = empty_colmajor(k, n, torch.float64, dev)
    rc = _lib.load().trqrcp_truncate(h.ptr, prec, m, n, k, b, p, _ptr(A), ld(A), _ptr(Omega),
                                     ld(Omega), _ptr(jpvt), _ptr(Y), ld(Y), _ptr(T), ld(T),
                                     _ptr(R), ld(R))
    _check("trqrcp_truncate", rc, h)
    return jpvt, Y, T, R


def tuxv_svd(A, Omega, b, p, k, handle=None, jmax=1, sigma=False):
    """TUXV (Algorithm 6, jmax alternations).  Returns (U, X, V, jpvt) with
    A ~ U X V^T (X upper for odd jmax, lower for even); with sigma=True also the
    singular values of X (largest first, computed on the device) as a fifth item."""
    h = handle or default_handle(A.device.index)
    m, n = A.shape
    dev = A.device
    prec = _DT[A.dtype]
    U = empty_colmajor(m, k, torch.float64, dev)
    X = empty_colmajor(k, k, torch.float64, dev)
    V = empty_colmajor(n, k, torch.float64, dev)
    jpvt = torch.empty(max(n, 1), dtype=torch.int64, device=dev)[:n]
    sv = torch.empty(max(k, 1), dtype=torch.float64, device=dev)[:k] if sigma else None
    if jmax == 1:
        rc = _lib.load().tuxv_svd(h.ptr, prec, m, n, k, b, p, _ptr(A), ld(A), _ptr(Omega),
                                  ld(Omega), _ptr(U), ld(U), _ptr(X), ld(X), _ptr(V), ld(V),
                                  _ptr(jpvt), _ptr(sv))
    else:
        rc = _lib.load().tuxv_svd_iter(h.ptr, prec, m, n, k, b, p, _ptr(A), ld(A), _ptr(Omega),
                                       ld(Omega), _ptr(U), ld(U), _ptr(X), ld(X), _ptr(V), ld(V),
                                       _ptr(jpvt), _ptr(sv), int(jmax))
    _check("tuxv_svd", rc, h)
    return (U, X, V, jpvt, sv) if sigma else (U, X, V, jpvt)


def singular_values(X, handle=None):
    """Singular values (largest first) of the square float64 device matrix X."""
    h = handle or default_handle(X.device.index)
    k = X.shape[0]
    if X.shape[1] != k:
        raise ValueError("X must be square")
    sv = torch.empty(max(k, 1), dtype=torch.float64, device=X.device)[:k]
    rc = _lib.load().rq_singular_values(h.ptr, k, _ptr(X), ld(X), _ptr(sv))
    _check("rq_singular_values", rc, h)
    return sv


def sketch(Omega, A, handle=None):
    """B = Omega A (ell x n, float64) on the device."""
    h = handle or default_handle(A.device.index)
    ell, m = Omega.shape
    n = A.shape[1]
    B = empty_colmajor(ell, n, torch.float64, A.device)
    rc = _lib.load().rq_sketch(h.ptr, _DT[A.dtype], ell, m, n, _ptr(Omega), ld(Omega), _ptr(A),
                               ld(A), _ptr(B), ld(B))
    _check("rq_sketch", rc, h)
    return B


def sample_qrcp(B, steps, handle=None):
    """QRCP(B, steps) in place on the sample B; returns perm (final <- input position)."""
    h = handle or default_handle(B.device.index)
    ell, n = B.shape
    perm = torch.empty(max(n, 1), dtype=torch.int64, device=B.device)[:n]
    rc = _lib.load().rq_sample_qrcp(h.ptr, ell, n, steps, _ptr(B), ld(B), _ptr(perm))
    _check("rq_sample_qrcp", rc, h)
    return perm


def sample_qrcp_noalloc(B, steps, perm, handle=None):
    """sample_qrcp without any device allocation: the library's static scratch
    array holds the exchange records and ``perm`` (int64, n) is caller-provided."""
    h = handle or default_handle(B.device.index)
    ell, n = B.shape
    rc = _lib.load().rq_sample_qrcp_noalloc(h.ptr, ell, n, steps, _ptr(B), ld(B), _ptr(perm))
    _check("rq_sample_qrcp_noalloc", rc, h)
    return perm


# ----------------------------------------------------------------------------- serving
def serve_route(prec, m, n, k, tol):
    """The arithmetic (RQ_FP64 or RQ_MIXED_BF16) the server runs such a request in."""
    return _lib.load().rq_serve_route(int(prec), m, n, k, float(tol))


def pinned_empty(shape, dtype):
    """Page-locked host array in column-major order (asynchronous copies)."""
    tdt = {np.float32: torch.float32, np.float64: torch.float64, np.int64: torch.int64}[dtype]
    if len(shape) == 2:
        t = torch.empty((shape[1], shape[0]), dtype=tdt, pin_memory=True).t()
    else:
        t = torch.empty(shape, dtype=tdt, pin_memory=True)
    return t.numpy()


class Server:
    """Continuous-batching server over rq_serve_* (requests in host memory)."""

    def __init__(self, budget_bytes, slots, max_m, max_n, max_k, max_ell, device=0):
        lib = _lib.load()
        self.ptr = ctypes.c_void_p()
        _check("rq_serve_start", lib.rq_serve_start(device, int(budget_bytes), slots, max_m, max_n,
                                                    max_k, max_ell, ctypes.byref(self.ptr)))
        self._keep = {}

    def submit(self, op, A, Omega, b, p, k, outputs=True, tol=None, sigma=False):
        """A, Omega: column-major host arrays.  float64 A runs in FP64; float32 A
        runs on BF16 MFMA, or, with ``tol`` (the relative error the request
        needs), in whichever arithmetic rq_serve_route picks (RQ_AUTO).  With
        sigma=True a TUXV request also returns the singular values of X."""
        lib = _lib.load()
        m, n = A.shape
        if not A.flags.f_contiguous or not Omega.flags.f_contiguous:
            raise ValueError("A and Omega must be column-major (Fortran order)")
        if A.dtype == np.float64:
            prec = RQ_FP64
        else:
            prec = _lib.RQ_AUTO if tol is not None else RQ_MIXED_BF16
        outs = None
        if outputs:
            if op == _lib.RQ_OP_TRQRCP:
                outs = (pinned_empty((n,), np.int64), pinned_empty((m, k), np.float64),
                        pinned_empty((k, k), np.float64), pinned_empty((k, n), np.float64))
            else:
                outs = (pinned_empty((n,), np.int64), pinned_empty((m, k), np.float64),
                        pinned_empty((k, k), np.float64), pinned_empty((n, k), np.float64))
        sv = pinned_empty((k,), np.float64) if (sigma and op == _lib.RQ_OP_TUXV) else None
        req = _lib.Request(op, prec, m, n, k, b, p, A.ctypes.data, Omega.ctypes.data,
                           outs[0].ctypes.data if outs else None,
                           outs[1].ctypes.data if outs else None,
                           outs[2].ctypes.data if outs else None,
                           outs[3].ctypes.data if outs else None,
                           sv.ctypes.data if sv is not None else None,
                           float(tol) if tol is not None else 0.0)
        rid = ctypes.c_uint64()
        rc = lib.rq_serve_submit(self.ptr, ctypes.byref(req), ctypes.byref(rid))
        if rc != 0:
            raise RQError("rq_serve_submit", rc)
        self._keep[rid.value] = (A, Omega, outs, sv)
        return rid.value

    def _result(self, fn, rid):
        res = _lib.Result()
        _check(fn.__name__, fn(self.ptr, rid, ctypes.byref(res)))
        d = {f: getattr(res, f) for f, _ in _lib.Result._fields_}
        keep = self._keep.get(rid, (None, None, None, None))
        d["outputs"] = keep[2]
        d["sigma"] = keep[3]
        return d

    def poll(self, rid):
        return self._result(_lib.load().rq_serve_poll, rid)

    def wait(self, rid):
        return self._result(_lib.load().rq_serve_wait, rid)

    def stats(self):
        c, pb, pr = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check("rq_serve_stats", _lib.load().rq_serve_stats(self.ptr, ctypes.byref(c),
                                                             ctypes.byref(pb), ctypes.byref(pr)))
        return {"completed": c.value, "peak_bytes": pb.value, "peak_running": pr.value}

    def release(self, rid):
        """Drop the binding's references to a finished request's host buffers."""
        self._keep.pop(rid, None)

    def stop(self):
        if self.ptr:
            _check("rq_serve_stop", _lib.load().rq_serve_stop(self.ptr))
            self.ptr = ctypes.c_void_p()
