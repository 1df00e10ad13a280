"""Host-side checks of the C ABI: libmbh.so loads and exports every entry
point declared in include/mbh.h; the binding rejects bad shapes before any
device call.  No kernel runs here."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2005_01827_amd import mbh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mbh.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mbh_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_surface():
    assert sorted(mbh.EXPORTED) == declared_functions()


def test_library_exports_every_declared_symbol():
    if not os.path.exists(mbh.LIB_PATH):
        from paper_2005_01827_amd import build
        build.build(force=False)
    lib = ctypes.CDLL(mbh.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", mbh.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\sT\s(mbh_\w+)", out.stdout))
    assert set(declared_functions()) <= exported


def test_version_and_error_text_without_gpu():
    L = mbh.load_library()
    assert L.mbh_version() >= 100
    assert L.mbh_last_error(None) == b"mbh: null context"


def test_create_rejects_bad_descriptors_without_touching_the_gpu():
    L = mbh.load_library()
    n = 64
    data = np.zeros((3, n, 2))
    psd = np.ones((3, n))

    def desc(**kw):
        d = mbh.CtxDesc()
        d.df, d.k0, d.n = 1e-4, 10, n
        d.data = data.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.psd = psd.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.n_modes = 1
        d.modes[0][0], d.modes[0][1] = 2, 2
        d.n_sparse, d.t0, d.precision, d.max_batch = 32, 0.0, 0, 4
        for k, v in kw.items():
            setattr(d, k, v)
        return d

    h = ctypes.c_void_p()
    for bad in (dict(df=0.0), dict(k0=0), dict(n=2), dict(n_modes=0), dict(n_modes=7), dict(n_sparse=3),
                dict(max_batch=0), dict(precision=5), dict(t0=float("nan"))):
        assert L.mbh_ctx_create(ctypes.byref(desc(**bad)), ctypes.byref(h)) == mbh.MBH_EINVAL
        assert not h.value
    d = desc()
    d.modes[0][0], d.modes[0][1] = 5, 5
    assert L.mbh_ctx_create(ctypes.byref(d), ctypes.byref(h)) == mbh.MBH_EINVAL
    psd[1, 3] = -1.0
    assert L.mbh_ctx_create(ctypes.byref(desc()), ctypes.byref(h)) == mbh.MBH_EINVAL
    psd[1, 3] = 1.0
    assert L.mbh_ctx_create(None, ctypes.byref(h)) == mbh.MBH_EINVAL
    for fn in ("mbh_response",):
        assert getattr(L, fn)(None, 1, None) == mbh.MBH_EINVAL
    assert L.mbh_loglike_batch(None, None, 1, None, None) == mbh.MBH_EINVAL


def test_binding_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2005_01827_amd import inputs
    w = inputs.small_config(1)
    with pytest.raises(RuntimeError):
        mbh.Likelihood(w.grid, np.zeros((3, w.grid.n), complex), inputs.psd_aet(w.grid.freqs), w.modes)
