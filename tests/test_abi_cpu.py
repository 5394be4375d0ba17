"""The C ABI without a GPU: the library loads, exports every function the
header declares, sizes its workspace, and rejects invalid arguments before
touching a device."""

import ctypes
import os
import re

import pytest

from paper_1304_2272_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gwas.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gwas_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libgwas.so not built")
    return binding.load()


def test_header_matches_binding():
    assert _declared() == sorted(binding.FUNCTIONS)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_workspace_bytes(lib):
    w = lib.gwas_workspace_bytes(1000, 4, 1, 0, 0, 0)
    n_pad = 1024
    assert w >= 2 * n_pad * n_pad * 8               # L and its inverse
    # the float32 path adds a float32 copy of the inverse factor
    assert lib.gwas_workspace_bytes(1000, 4, 1, 0, 1, 0) >= 2 * n_pad * n_pad * 8 + n_pad * n_pad * 4
    # int8 dosages need an eighth of the float64 staging buffers
    assert lib.gwas_workspace_bytes(1000, 4, 1, 0, 0, 1) < w
    assert lib.gwas_workspace_bytes(1024, 4, 1, 0, 0, 0) == w       # same padded order
    # invalid sizes give 0
    for args in [(3, 4, 1, 0, 0, 0), (100, 1, 1, 0, 0, 0), (100, 21, 1, 0, 0, 0),
                 (100, 4, 0, 0, 0, 0), (100, 4, 1, -1, 0, 0), (100, 4, 1, 0, 7, 0),
                 (100, 4, 1, 0, 0, 5), (100, 4, 257, 0, 0, 0)]:
        assert lib.gwas_workspace_bytes(*args) == 0, args


def _desc(n=16, p=3, t=1, **kw):
    import numpy as np
    M = np.eye(n)
    XL = np.ones((p - 1, n))
    Y = np.ones((t, n))
    d = binding.Desc(n=n, p=p, t=t, M=M.ctypes.data, ldm=n, XL=XL.ctypes.data, ldxl=n,
                     Y=Y.ctypes.data, ldy=n, inputs_on_device=0, precision=0, x_dtype=0,
                     device=0, dev_block=0, workspace=None, workspace_bytes=0, stream=None)
    for k, v in kw.items():
        setattr(d, k, v)
    return d, (M, XL, Y)


@pytest.mark.parametrize("field,value", [
    ("n", 2), ("p", 1), ("p", 21), ("t", 0), ("ldm", 5), ("ldxl", 5), ("ldy", 5),
    ("precision", 9), ("x_dtype", 3), ("M", None), ("XL", None), ("Y", None),
    ("dev_block", -5),
])
def test_init_rejects_invalid_before_device(lib, field, value):
    d, keep = _desc(**{field: value})
    h = ctypes.c_void_p(123)
    assert lib.gwas_init(ctypes.byref(h), ctypes.byref(d)) == 1   # GWAS_E_INVALID
    assert h.value is None


def test_init_without_device_reports_no_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    d, keep = _desc()
    h = ctypes.c_void_p()
    assert lib.gwas_init(ctypes.byref(h), ctypes.byref(d)) == 4   # GWAS_E_NO_DEVICE
    assert h.value is None


def test_null_context_calls(lib):
    assert lib.gwas_free(None) == 0
    assert lib.gwas_stream_block(None, None, 0, 0, None, 0, None, None) == 7
    assert lib.gwas_info(None) == -1
    assert lib.gwas_set_timing(None, 1) == 7
    assert lib.gwas_test_inject_fault(None, 1) == 7
    assert lib.gwas_strerror(2).decode().startswith("M is not positive definite")
    assert lib.gwas_strerror(12345).decode() == "unknown status"


def test_peak_probe_validates_before_device(lib):
    out = ctypes.c_double(-1.0)
    assert lib.gwas_peak_probe(7, 0, 100, ctypes.byref(out)) == 1      # bad kind
    assert lib.gwas_peak_probe(0, 0, 0, ctypes.byref(out)) == 1        # iters < 1
    assert lib.gwas_peak_probe(0, 0, 100, None) == 1                   # no result pointer
    assert out.value == -1.0
    import torch
    if not torch.cuda.is_available():
        assert lib.gwas_peak_probe(0, 0, 100, ctypes.byref(out)) == 4  # GWAS_E_NO_DEVICE
