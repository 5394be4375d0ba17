"""Thin ctypes binding over the C ABI declared in ``include/gwas.h``.

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when ``libgwas.so`` has not been built; there
is no fallback path.

Array conventions on the Python side (all float64 unless stated):
  M   (n, n) symmetric.  The library reads the triangle that is lower in
      column-major order, i.e. the upper triangle of a C-ordered array.
  XL  (n, p-1) covariates, Y (n,) or (n, t) phenotypes.
  XR  (m, n) C-ordered, one row per SNP (the column-major n x m matrix whose
      column i is SNP i); float64 or int8 per ``x_dtype``.
  b   (m, t, p) output, SNP coefficient last; var (m,); info (m,) int32.
numpy arrays are host memory; torch tensors may live on the GPU.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgwas.so")

GWAS_OK = 0
ERRORS = {1: "GWAS_E_INVALID", 2: "GWAS_E_NOT_SPD", 3: "GWAS_E_RANK_XL", 4: "GWAS_E_NO_DEVICE",
          5: "GWAS_E_HIP", 6: "GWAS_E_OOM", 7: "GWAS_E_STATE", 8: "GWAS_E_WORKSPACE"}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "int8": 3, "bf16x3": 4}
X_DTYPES = {"f64": 0, "i8": 1}

FUNCTIONS = ("gwas_workspace_bytes", "gwas_init", "gwas_stream_block", "gwas_free",
             "gwas_strerror", "gwas_info", "gwas_last_error", "gwas_set_timing",
             "gwas_kernel_time", "gwas_query", "gwas_stream_group", "gwas_autotune",
             "gwas_backward_begin", "gwas_backward_block", "gwas_backward_end", "gwas_peak_probe",
             "gwas_test_inject_fault", "gwas_stream_block_async", "gwas_stream_wait",
             "gwas_stream_block_noalloc", "gwas_workspace_bytes_band")
GROUP_GRAPH = 1


class Desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("p", ctypes.c_int32), ("t", ctypes.c_int32),
        ("M", ctypes.c_void_p), ("ldm", ctypes.c_int64),
        ("XL", ctypes.c_void_p), ("ldxl", ctypes.c_int64),
        ("Y", ctypes.c_void_p), ("ldy", ctypes.c_int64),
        ("inputs_on_device", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("x_dtype", ctypes.c_int32), ("device", ctypes.c_int32),
        ("dev_block", ctypes.c_int64),
        ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
        ("stream", ctypes.c_void_p),
        ("slices", ctypes.c_int32),
        ("band", ctypes.c_int64),
    ]


class GwasError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")


_lib = None


def load():
    """Load ``libgwas.so`` and declare its signatures (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # One HIP runtime per process: torch ships its own libamdhip64 with the
    # same soname, so loading torch first makes the library bind to it and
    # device pointers and streams from torch stay valid in the library.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.gwas_workspace_bytes.restype = ctypes.c_size_t
    L.gwas_workspace_bytes.argtypes = [i64, i32, i32, i64, i32, i32]
    L.gwas_workspace_bytes_band.restype = ctypes.c_size_t
    L.gwas_workspace_bytes_band.argtypes = [i64, i32, i32, i64, i64, i64, i32]
    L.gwas_init.restype = ctypes.c_int
    L.gwas_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Desc)]
    L.gwas_stream_block.restype = ctypes.c_int
    L.gwas_stream_block.argtypes = [vp, vp, i64, i64, vp, i64, vp, vp]
    L.gwas_free.restype = ctypes.c_int
    L.gwas_free.argtypes = [vp]
    L.gwas_strerror.restype = ctypes.c_char_p
    L.gwas_strerror.argtypes = [ctypes.c_int]
    L.gwas_info.restype = i64
    L.gwas_info.argtypes = [vp]
    L.gwas_last_error.restype = ctypes.c_char_p
    L.gwas_last_error.argtypes = [vp]
    L.gwas_set_timing.restype = ctypes.c_int
    L.gwas_set_timing.argtypes = [vp, i32]
    L.gwas_kernel_time.restype = ctypes.c_int
    L.gwas_kernel_time.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(i64)]
    L.gwas_query.restype = ctypes.c_int
    L.gwas_query.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.gwas_stream_group.restype = ctypes.c_int
    L.gwas_stream_group.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(i64), i64,
                                    ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(vp),
                                    ctypes.POINTER(vp), i32]
    L.gwas_autotune.restype = ctypes.c_int
    L.gwas_autotune.argtypes = [vp, vp, i64, i64, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.gwas_backward_begin.restype = ctypes.c_int
    L.gwas_backward_begin.argtypes = [vp]
    L.gwas_backward_block.restype = ctypes.c_int
    L.gwas_backward_block.argtypes = [vp, vp, i64, i64, vp, i64, vp, vp, vp, i64, vp]
    L.gwas_backward_end.restype = ctypes.c_int
    L.gwas_backward_end.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.gwas_peak_probe.restype = ctypes.c_int
    L.gwas_peak_probe.argtypes = [i32, i32, i64, ctypes.POINTER(ctypes.c_double)]
    L.gwas_test_inject_fault.restype = ctypes.c_int
    L.gwas_test_inject_fault.argtypes = [vp, i64]
    L.gwas_stream_block_async.restype = ctypes.c_int
    L.gwas_stream_block_async.argtypes = [vp, vp, i64, i64, vp, i64, vp, vp]
    L.gwas_stream_wait.restype = ctypes.c_int
    L.gwas_stream_wait.argtypes = [vp]
    L.gwas_stream_block_noalloc.restype = ctypes.c_int
    L.gwas_stream_block_noalloc.argtypes = [vp, vp, i64, i64, vp, i64, vp, vp]
    _lib = L
    return L


def peak_probe(precision, device=0, iters=20000):
    """Measured matrix-core rate (operations/s) of the instruction the
    triangular product of ``precision`` runs (see ``gwas_peak_probe``)."""
    L = load()
    out = ctypes.c_double()
    rc = L.gwas_peak_probe(PRECISIONS[precision], device, iters, ctypes.byref(out))
    if rc:
        raise GwasError(rc, L.gwas_strerror(rc).decode())
    return out.value


def workspace_bytes(n, p, t=1, dev_block=0, precision="fp64", x_dtype="f64"):
    return load().gwas_workspace_bytes(n, p, t, dev_block, PRECISIONS[precision], X_DTYPES[x_dtype])


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr_ld(a, want_dtype, what):
    """(pointer, leading dimension, keepalive, on_device) of a column-major view.

    ``a`` is given row-major as (cols, rows): rows of ``a`` are columns of the
    column-major matrix handed to the library.
    """
    if _is_torch(a):
        import torch
        tdt = {np.float64: torch.float64, np.int8: torch.int8}[want_dtype]
        if a.dtype != tdt:
            raise TypeError(f"{what}: expected {tdt}, got {a.dtype}")
        if a.dim() == 1:
            a = a.reshape(1, -1)
        if a.stride(-1) != 1:
            a = a.contiguous()
        # a single row keeps its stride when that is a valid leading dimension
        ld = a.stride(0) if (a.shape[0] > 1 or a.stride(0) >= a.shape[1]) else a.shape[1]
        return a.data_ptr(), ld, a, a.is_cuda
    a = np.asarray(a)
    if a.dtype != want_dtype:
        raise TypeError(f"{what}: expected {np.dtype(want_dtype)}, got {a.dtype}")
    if a.ndim == 1:
        a = a.reshape(1, -1)
    if a.strides[-1] != a.itemsize:
        a = np.ascontiguousarray(a)
    ld = a.strides[0] // a.itemsize
    if a.shape[0] == 1 and ld < a.shape[1]:
        ld = a.shape[1]
    return a.ctypes.data, ld, a, False


class GwasContext:
    """One factorisation of M and its derived constants, reused for every block."""

    def __init__(self, M, XL, Y, precision="fp64", x_dtype="f64", dev_block=0, device=0,
                 stream=None, slices=0, band=0):
        """M is (n, n), or with ``band`` = w >= 1 the lower band storage of a
        banded M as an (n, ldm) array, ldm >= w + 1: M[j, d] = M(j + d, j)."""
        L = load()
        self._lib = L
        self.precision = precision
        self.x_dtype = x_dtype
        self._pending = []
        dev = _is_torch(M) and M.is_cuda
        if dev:
            import torch
            n = M.shape[0]
            XLt = XL.reshape(n, -1).t().contiguous()
            Yt = (Y.reshape(n, 1) if Y.dim() == 1 else Y).t().contiguous()
            Mk = M.contiguous()
            if stream is None:
                stream = torch.cuda.current_stream(M.device).cuda_stream
            keep = (Mk, XLt, Yt)
            mp, xlp, yp = Mk.data_ptr(), XLt.data_ptr(), Yt.data_ptr()
            p = XLt.shape[0] + 1
            t = Yt.shape[0]
        else:
            M = np.ascontiguousarray(np.asarray(M, dtype=np.float64))
            n = M.shape[0]
            XLt = np.ascontiguousarray(np.asarray(XL, dtype=np.float64).reshape(n, -1).T)
            Yv = np.asarray(Y, dtype=np.float64)
            Yt = np.ascontiguousarray((Yv.reshape(n, 1) if Yv.ndim == 1 else Yv).T)
            keep = (M, XLt, Yt)
            mp, xlp, yp = M.ctypes.data, XLt.ctypes.data, Yt.ctypes.data
            p = XLt.shape[0] + 1
            t = Yt.shape[0]
        self.n, self.p, self.t = n, p, t
        ldm = keep[0].shape[1] if band else n
        d = Desc(n=n, p=p, t=t, M=mp, ldm=ldm, XL=xlp, ldxl=n, Y=yp, ldy=n,
                 inputs_on_device=1 if dev else 0, precision=PRECISIONS[precision],
                 x_dtype=X_DTYPES[x_dtype], device=device, dev_block=dev_block,
                 workspace=None, workspace_bytes=0, stream=stream, slices=slices, band=band)
        h = ctypes.c_void_p()
        rc = L.gwas_init(ctypes.byref(h), ctypes.byref(d))
        del keep
        self._h = h
        if rc != GWAS_OK:
            info = L.gwas_info(h) if h.value else 0
            msg = L.gwas_last_error(h).decode() if h.value else L.gwas_strerror(rc).decode()
            if h.value:
                L.gwas_free(h)
                self._h = ctypes.c_void_p()
            err = GwasError(rc, msg)
            err.info = info
            raise err

    def _check(self, rc):
        if rc != GWAS_OK:
            msg = self._lib.gwas_last_error(self._h).decode() if self._h.value else ""
            raise GwasError(rc, msg or self._lib.gwas_strerror(rc).decode())

    def stream_block(self, XR, out=None):
        """Solve Eq. (1) for every SNP row of XR; returns (b, var, info)."""
        xdt = np.int8 if self.x_dtype == "i8" else np.float64
        xp, ldx, keep, xdev = _ptr_ld(XR, xdt, "XR")
        m = XR.shape[0] if XR.ndim == 2 else 1
        pt = self.p * self.t
        if out is not None:
            b, var, info = out
        elif xdev:
            import torch
            b = torch.empty((m, self.t, self.p), dtype=torch.float64, device=XR.device)
            var = torch.empty(m, dtype=torch.float64, device=XR.device)
            info = torch.empty(m, dtype=torch.int32, device=XR.device)
        else:
            b = np.empty((m, self.t, self.p))
            var = np.empty(m)
            info = np.empty(m, dtype=np.int32)
        ptr = (lambda a: a.data_ptr()) if _is_torch(b) else (lambda a: a.ctypes.data)
        rc = self._lib.gwas_stream_block(self._h, xp, ldx, m, ptr(b), pt,
                                         ptr(var) if var is not None else None,
                                         ptr(info) if info is not None else None)
        del keep
        self._check(rc)
        return b, var, info

    def stream_block_async(self, XR, out):
        """Queue a block and return at once (``gwas_stream_block_async``).
        ``out`` = (b, var, info) as for :meth:`stream_block`; XR and ``out``
        must stay unchanged until :meth:`wait`, and the binding keeps them
        alive until then."""
        xdt = np.int8 if self.x_dtype == "i8" else np.float64
        xp, ldx, keep, _ = _ptr_ld(XR, xdt, "XR")
        m = XR.shape[0] if XR.ndim == 2 else 1
        b, var, info = out
        ptr = (lambda a: a.data_ptr()) if _is_torch(b) else (lambda a: a.ctypes.data)
        rc = self._lib.gwas_stream_block_async(self._h, xp, ldx, m, ptr(b), self.p * self.t,
                                               ptr(var) if var is not None else None,
                                               ptr(info) if info is not None else None)
        self._pending.append((keep, XR, out))
        self._check(rc)

    def stream_block_noalloc(self, XR, out):
        """Queue the block on the context's stream without any allocation
        (``gwas_stream_block_noalloc``); XR and ``out`` = (b, var, info) are
        device tensors, valid once that stream has reached this point."""
        xp, ldx, keep, xdev = _ptr_ld(XR, np.int8 if self.x_dtype == "i8" else np.float64, "XR")
        m = XR.shape[0] if XR.ndim == 2 else 1
        b, var, info = out
        if not (xdev and all(a is None or (_is_torch(a) and a.is_cuda) for a in out)):
            raise TypeError("stream_block_noalloc takes device tensors only")
        if keep.data_ptr() != XR.data_ptr():
            raise ValueError("XR must have unit stride along n: the call copies nothing")
        rc = self._lib.gwas_stream_block_noalloc(self._h, xp, ldx, m, b.data_ptr(), self.p * self.t,
                                                 var.data_ptr() if var is not None else None,
                                                 info.data_ptr() if info is not None else None)
        self._check(rc)

    def wait(self):
        """Wait for the blocks queued by :meth:`stream_block_async`."""
        rc = self._lib.gwas_stream_wait(self._h)
        self._pending = []
        self._check(rc)

    def _outputs(self, m, xdev, device):
        if xdev:
            import torch
            return (torch.empty((m, self.t, self.p), dtype=torch.float64, device=device),
                    torch.empty(m, dtype=torch.float64, device=device),
                    torch.empty(m, dtype=torch.int32, device=device))
        return np.empty((m, self.t, self.p)), np.empty(m), np.empty(m, dtype=np.int32)

    def autotune(self, XR, cols=None):
        """Time every tile shape and schedule row group on the first ``cols``
        SNPs of XR; keep the fastest.  Returns (shape, row group)."""
        xdt = np.int8 if self.x_dtype == "i8" else np.float64
        xp, ldx, keep, _ = _ptr_ld(XR, xdt, "XR")
        cols = XR.shape[0] if cols is None else cols
        best, rg = ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.gwas_autotune(self._h, xp, ldx, cols, ctypes.byref(best), ctypes.byref(rg)))
        del keep
        return best.value, rg.value

    def backward_begin(self):
        """Start a reverse pass (forms M^-1 and W on the first call)."""
        self._check(self._lib.gwas_backward_begin(self._h))

    def backward_block(self, XR, b, var, info, gb, gvar=None):
        """Add one block's contribution: XR as given to stream_block, (b, var,
        info) its outputs, gb = dl/db (m, p) and gvar = dl/dvar (m,)."""
        xdt = np.int8 if self.x_dtype == "i8" else np.float64
        xp, ldx, keep, _ = _ptr_ld(XR, xdt, "XR")
        m = XR.shape[0] if XR.ndim == 2 else 1
        arrs = [b, var, info, gb] + ([gvar] if gvar is not None else [])
        conv = []
        for a in arrs:
            if _is_torch(a):
                conv.append(a.contiguous())
            else:
                conv.append(np.ascontiguousarray(a))
        ptr = lambda a: a.data_ptr() if _is_torch(a) else a.ctypes.data
        bb, vv, ii, gg = conv[:4]
        gv = conv[4] if gvar is not None else None
        rc = self._lib.gwas_backward_block(self._h, xp, ldx, m, ptr(bb), self.p, ptr(vv), ptr(ii), ptr(gg),
                                           self.p, ptr(gv) if gv is not None else None)
        del keep, conv
        self._check(rc)

    def backward_end(self, gy=None):
        """(dl/dy, tr Mbar, <Mbar, M>); dl/dy goes into ``gy`` if given."""
        if gy is None:
            gy = np.empty(self.n)
        tr = ctypes.c_double()
        ip = ctypes.c_double()
        ptr = gy.data_ptr() if _is_torch(gy) else gy.ctypes.data
        self._check(self._lib.gwas_backward_end(self._h, ptr, ctypes.byref(tr), ctypes.byref(ip)))
        return gy, tr.value, ip.value

    def set_timing(self, on=True):
        self._check(self._lib.gwas_set_timing(self._h, 1 if on else 0))

    def kernel_time(self):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        cols = ctypes.c_int64()
        self._check(self._lib.gwas_kernel_time(self._h, ctypes.byref(n), ctypes.byref(ms),
                                               ctypes.byref(cols)))
        return n.value, ms.value, cols.value

    def query(self):
        npad = ctypes.c_int64()
        blk = ctypes.c_int64()
        dev = ctypes.c_int32()
        self._check(self._lib.gwas_query(self._h, ctypes.byref(npad), ctypes.byref(blk),
                                         ctypes.byref(dev)))
        return {"n_pad": npad.value, "dev_block": blk.value, "device": dev.value}

    def inject_fault(self, k):
        """Test hook: the k-th HIP status later calls check is reported as a
        failure (0 turns it off); see gwas_test_inject_fault."""
        self._check(self._lib.gwas_test_inject_fault(self._h, int(k)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.gwas_free(self._h)   # waits for queued blocks before it releases anything
            self._h = ctypes.c_void_p()
        self._pending = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def stream_group(ctxs, XRs, graph=False):
    """Solve the same SNP positions for several contexts (cohorts) in grouped
    launches; returns a list of (b, var, info) per context."""
    L = load()
    n = len(ctxs)
    if len(XRs) != n or n == 0:
        raise ValueError("one dosage block per context")
    xdt = np.int8 if ctxs[0].x_dtype == "i8" else np.float64
    ptrs, lds, keeps, outs = [], [], [], []
    m = XRs[0].shape[0]
    for c, X in zip(ctxs, XRs):
        if X.shape[0] != m:
            raise ValueError("all blocks must hold the same SNP positions")
        xp, ldx, keep, xdev = _ptr_ld(X, xdt, "XR")
        ptrs.append(xp)
        lds.append(ldx)
        keeps.append(keep)
        outs.append(c._outputs(m, xdev, X.device if xdev else None))
    ptr = (lambda a: a.data_ptr()) if _is_torch(outs[0][0]) else (lambda a: a.ctypes.data)
    VP = ctypes.c_void_p
    I64 = ctypes.c_int64
    hs = (VP * n)(*[c._h.value for c in ctxs])
    xs = (VP * n)(*ptrs)
    lx = (I64 * n)(*lds)
    bs = (VP * n)(*[ptr(o[0]) for o in outs])
    lb = (I64 * n)(*[c.p * c.t for c in ctxs])
    vs = (VP * n)(*[ptr(o[1]) for o in outs])
    ins = (VP * n)(*[ptr(o[2]) for o in outs])
    rc = L.gwas_stream_group(hs, n, xs, lx, m, bs, lb, vs, ins, GROUP_GRAPH if graph else 0)
    del keeps
    if rc != GWAS_OK:
        raise GwasError(rc, L.gwas_last_error(ctxs[0]._h).decode())
    return outs
