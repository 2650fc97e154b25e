"""C ABI: the library loads, exports every declared symbol, and rejects bad
arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
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
    assert o.max_iter == 500 and o.lbfgs_m == 40


def test_create_rejects_bad_config_without_device():
    from paper_1502_04993_amd import _lib
    lib = _lib.load()
    out = ctypes.c_void_p()
    for kw in (dict(n_neurons=0), dict(n_bins=0), dict(dt=0.0), dict(dt=float("nan")),
               dict(precision=7), dict(tile_n=100), dict(chunk_bins=-1), dict(trace=3),
               dict(precision=3, trace=2),  # FP8 exists only on the resident trace
               dict(time_mode=2), dict(time_mode=1, precision=3)):
        args = dict(n_neurons=10, n_bins=100, dt=0.001, chunk_bins=0, precision=1, device=0,
                    stream=None, tile_n=0, trace=0, time_mode=0)
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
    n = ctypes.c_size_t(0)
    assert lib.glmr_get_state(None, None, ctypes.byref(n)) == _lib.GLMR_EINVAL
    assert lib.glmr_set_state(None, b"GLMRST02", 8) == _lib.GLMR_EINVAL
    o = _lib.glmr_fit_opts()
    lib.glmr_fit_defaults(ctypes.byref(o))
    assert o.resume == 0 and o.keep_history == 0  # a fit starts afresh unless asked otherwise


def test_null_context_event_calls():
    from paper_1502_04993_amd import _lib
    lib = _lib.load()
    assert lib.glmr_set_spike_times(None, None, None, 0, 0.0, 1.0, 0.0, 0) == _lib.GLMR_EINVAL


def test_event_slots_counts_and_rejections():
    import paper_1502_04993_amd as G
    t = np.array([0.1, 0.2, 0.5])
    # gaps 0.1, 0.1, 0.3 (two slots), tail 0.5 (ceil(0.5 / 0.15) = 4 slots)
    assert G.glmr_event_slots(t, 0.0, 1.0, 0.15) == 1 + 1 + 2 + 4
    # no split needed: one slot from T0 and one per event
    assert G.glmr_event_slots(t, 0.0, 1.0, 10.0) == 4
    assert G.glmr_event_slots(np.array([]), 0.0, 1.0, 0.3) == 4
    # default max_gap 4 (T1 - T0) / (q + 1) = 1: no gap above it here
    assert G.glmr_event_slots(t, 0.0, 1.0) == 4
    for bad in (np.array([0.3, 0.2]), np.array([-0.1]), np.array([1.0]), np.array([np.nan])):
        with pytest.raises(G.GlmrError):
            G.glmr_event_slots(bad, 0.0, 1.0, 0.1)
    with pytest.raises(G.GlmrError):
        G.glmr_event_slots(t, 1.0, 1.0, 0.1)
    with pytest.raises(G.GlmrError):
        G.glmr_event_slots(t, 0.0, 1.0, 1e-12)  # more than 1e9 slots per window
