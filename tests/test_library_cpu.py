"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol include/enufft.h declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2606_21278_amd as enf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "enufft.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(enufft_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["enufft_plan", "enufft_type1_batched", "enufft_ems", "enufft_type1_adjoint", "enufft_destroy",
              "enufft_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = enf.load_library()
    for n in _declared():
        assert hasattr(L, n), n
    assert set(_declared()) == set(enf.EXPORTS)
    assert L.enufft_version().startswith(b"enufft-gfx950")


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ImportError):
        enf.load_library(str(tmp_path / "nope.so"))


def _plan(n_cells=2, offsets=None, windows=True, **kw):
    L = enf.load_library()
    o = enf.Opts()
    assert L.enufft_default_opts(ctypes.byref(o)) == enf.OK
    for k, v in kw.items():
        if k == "n_modes":
            o.n_modes[0], o.n_modes[1] = v
        else:
            setattr(o, k, v)
    off = np.array(offsets if offsets is not None else [0, 5, 9][: n_cells + 1], dtype=np.int64)
    w = (enf.Window * 4)(*[enf.Window(0.0, 0.0, 3.0)] * 4) if windows else None
    h = ctypes.c_void_p()
    st = L.enufft_plan(ctypes.byref(h), n_cells, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), w,
                       ctypes.byref(o), None)
    return st, h, L


def test_default_opts():
    L = enf.load_library()
    o = enf.Opts()
    assert L.enufft_default_opts(ctypes.byref(o)) == enf.OK
    assert (o.n_modes[0], o.n_modes[1], o.sigma, o.eps, o.precision) == (64, 64, 2.0, 1e-5, enf.F32)
    assert L.enufft_default_opts(None) == enf.EINVAL


@pytest.mark.parametrize("kw,code", [
    (dict(offsets=[0, 5, 3]), enf.EINVAL),                 # non-monotone offsets
    (dict(offsets=[1, 5, 9]), enf.EINVAL),                 # offsets[0] != 0
    (dict(n_modes=(0, 64)), enf.EINVAL),
    (dict(sigma=1.1), enf.EINVAL),
    (dict(eps=0.0), enf.EINVAL),
    (dict(eps=1e-7), enf.EEPS),                            # FP32 cannot reach 1e-7
    (dict(eps=1e-14, precision=enf.F64), enf.EEPS),
    (dict(precision=7), enf.EINVAL),
    (dict(window_kind=5), enf.EINVAL),
    (dict(windows=False), enf.EINVAL),                     # Hann needs windows
    (dict(kernel_width=40), enf.EINVAL),
    (dict(autotune=3), enf.EINVAL),                        # 0, 1 (raster trials) or 2 (unordered)
    (dict(autotune=-1), enf.EINVAL),
    (dict(n_modes=(2100, 64)), enf.EUNSUPPORTED),           # fine grid above 4096
])
def test_plan_argument_errors(kw, code):
    st, h, L = _plan(**kw)
    assert st == code
    assert h.value is None
    assert len(L.enufft_last_error(None)) > 0


def test_plan_null_pointers():
    L = enf.load_library()
    o = enf.Opts()
    L.enufft_default_opts(ctypes.byref(o))
    assert L.enufft_plan(None, 1, None, None, ctypes.byref(o), None) == enf.EINVAL
    h = ctypes.c_void_p()
    assert L.enufft_plan(ctypes.byref(h), 1, None, None, ctypes.byref(o), None) == enf.EINVAL
    off = np.array([0, 3], dtype=np.int64)
    assert L.enufft_plan(ctypes.byref(h), 1, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None, None,
                         None) == enf.EINVAL


def test_calls_on_null_plan_are_rejected():
    L = enf.load_library()
    assert L.enufft_type1_batched(None, None, None, None, None, None) == enf.EINVAL
    assert L.enufft_ems(None, None, None, None, None, None, None) == enf.EINVAL
    assert L.enufft_type1_adjoint(None, *([None] * 8)) == enf.EINVAL
    assert L.enufft_destroy(None) == enf.OK
    assert L.enufft_set_timing(None, 1) == enf.EINVAL


@pytest.mark.skipif(os.path.exists("/dev/kfd") and os.access("/dev/kfd", os.R_OK), reason="a GPU is present")
def test_valid_plan_without_gpu_reports_device_error():
    st, h, L = _plan()
    assert st == enf.EDEVICE
    assert b"gfx950" in L.enufft_last_error(None)
