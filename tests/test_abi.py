"""C ABI: the library loads, exports every declared symbol, and rejects bad
arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glmrec.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(glmr_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_1502_04993_amd import _lib
    lib = _lib.load()
    syms = declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(_lib.SIGNATURES)


def test_status_strings_and_defaults():
    import paper_1502_04993_amd as G
    assert G.glmr_status_string(0) == "ok"
    assert "invalid" in G.glmr_status_string(-1)
    o = G.glmr_fit_defaults()
    assert o.max_iter == 500 and o.lbfgs_m == 10


def test_create_rejects_bad_config_without_device():
    from paper_1502_04993_amd import _lib
    lib = _lib.load()
    out = ctypes.c_void_p()
    for kw in (dict(n_neurons=0), dict(n_bins=0), dict(dt=0.0), dict(dt=float("nan")),
               dict(precision=7), dict(tile_n=100), dict(chunk_bins=-1), dict(trace=3),
               dict(precision=3, trace=2)):  # FP8 exists only on the resident trace
        args = dict(n_neurons=10, n_bins=100, dt=0.001, chunk_bins=0, precision=1, device=0,
                    stream=None, tile_n=0, trace=0)
        args.update(kw)
        cfg = _lib.glmr_config(**args)
        assert lib.glmr_create(ctypes.byref(cfg), ctypes.byref(out)) == _lib.GLMR_EINVAL
        assert not out.value
    assert lib.glmr_create(None, ctypes.byref(out)) == _lib.GLMR_EINVAL
    lib.glmr_destroy(None)  # NULL-safe


def test_null_context_calls():
    from paper_1502_04993_amd import _lib
    lib = _lib.load()
    assert lib.glmr_set_kernel(None, 0.01) == _lib.GLMR_EINVAL
    assert lib.glmr_eval(None, None, None, None, None, None, 0) == _lib.GLMR_EINVAL
    assert lib.glmr_fit(None, None, None) == _lib.GLMR_EINVAL
