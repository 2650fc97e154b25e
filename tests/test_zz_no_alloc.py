"""glmr_set_kernel_noalloc: the per-tau set-up without device allocation
(its temporaries in the library's static scratch), called through the C ABI
and checked against glmr_set_kernel on the same recording (needs an MI355X).

Two calls in a row on one GPU, the second with a smaller recording (the
static scratch then holds the first call's contents).  The spike term's FP64
partial sums may be split over fewer time splits than glmr_set_kernel's, so
the two agree to the FP64 rounding of that sum: L and the gradient to 1e-12
relative (2-norm and element-wise) in every precision (the rest of the
evaluation is the same arithmetic on the same inputs).
"""
import ctypes

import numpy as np
import pytest

import synth
from parity_check import check

pytestmark = pytest.mark.gpu

SAME = dict(ll=1e-12, row=1e-12, grad=1e-12, gmax=1e-12)


def _G():
    import paper_1502_04993_amd as G
    return G


def _pair(rec, prec, tau_first, tau, **kw):
    """Context a: glmr_set_kernel(tau).  Context b: glmr_set_kernel(tau_first)
    (allocates the per-tau buffers), then glmr_set_kernel_noalloc(tau)."""
    G = _G()
    lib = G.L.load()
    a = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision=prec, **kw)
    b = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision=prec, **kw)
    for c in (a, b):
        c.set_spikes(rec.bins, rec.neurons)
    assert lib.glmr_set_kernel(a.handle, ctypes.c_double(tau)) == 0
    assert lib.glmr_set_kernel(b.handle, ctypes.c_double(tau_first)) == 0
    st = lib.glmr_set_kernel_noalloc(b.handle, ctypes.c_double(tau))
    assert st == 0, lib.glmr_last_error(b.handle)
    return a, b


@pytest.mark.parametrize("prec", ["bf16", "fp64", "fp8", "fp32"])
def test_noalloc_set_kernel_matches_set_kernel_twice(prec):
    # first call: N = 1000, 3e5 bins (carry segments 2 x 74 x 1024 x 16 B,
    # spike-term splits limited by the scratch); second: a smaller recording
    recs = [synth.config2(0, B=300_000), synth.balanced(N=70, B=20_000, seed=5)]
    for k, rec in enumerate(recs):
        a, b = _pair(rec, prec, 1.7 * rec.tau, rec.tau)
        J = rec.J
        for c in (a, b):
            c.set_params(J, rec.mu)
        ra, rb = a.eval(grad=True), b.eval(grad=True)
        assert a.get_params()[2] == b.get_params()[2] == rec.tau
        check(f"noalloc {prec} call {k} N={rec.n_neurons} B={rec.n_bins}", rb, ra, SAME)
        a.close()
        b.close()


def test_noalloc_set_kernel_event_grid_and_tau_caches():
    # the event grid (span maximum in the scratch) and the dL/dtau caches
    G = _G()
    rec = synth.balanced(N=150, B=12_000, in_frac=0.3, seed=241)
    times, neu = synth.event_times(rec, seed=5)
    a = G.Context.from_events(150, times, neu, 0.0, rec.T, precision="bf16")
    b = G.Context.from_events(150, times, neu, 0.0, rec.T, precision="bf16")
    a.set_kernel(rec.tau)
    b.set_kernel(2.0 * rec.tau)
    b.set_kernel_noalloc(rec.tau)
    for c in (a, b):
        c.set_params(rec.J, rec.mu)
    check("noalloc events", b.eval(grad=True), a.eval(grad=True), SAME)
    a.close()
    b.close()
    g = synth.balanced(N=60, B=8_000, seed=242)
    a, b = _pair(g, "fp64", 0.02, g.tau)
    for c in (a, b):
        c.set_params(g.J, g.mu)
        c.eval(want_tau=True)  # keeps the tau-derivative caches from now on
    a.set_kernel(0.013)
    b.set_kernel_noalloc(0.013)
    ra, rb = a.eval(grad=True, want_tau=True), b.eval(grad=True, want_tau=True)
    check("noalloc tau caches", rb, ra, SAME)
    assert abs(ra["gtau"] - rb["gtau"]) <= 1e-12 * abs(ra["gtau"])
    a.close()
    b.close()


def test_noalloc_set_kernel_refusals():
    G = _G()
    lib = G.L.load()
    rec = synth.balanced(N=40, B=5_000, seed=243)
    c = G.Context(40, 5_000, rec.dt, precision="fp64")
    c.set_spikes(rec.bins, rec.neurons)
    # before any glmr_set_kernel the per-tau buffers do not exist
    assert lib.glmr_set_kernel_noalloc(c.handle, ctypes.c_double(0.01)) == G.L.GLMR_ESTATE
    c.set_kernel(0.01)
    assert lib.glmr_set_kernel_noalloc(c.handle, ctypes.c_double(-1.0)) == G.L.GLMR_EINVAL
    assert lib.glmr_set_kernel_noalloc(c.handle, ctypes.c_double(0.0005)) == G.L.GLMR_EINVAL  # tau < dt
    c.close()
    # a recording whose set-up needs more than the static scratch: one time
    # split of the spike term alone is 6144^2 x 8 B = 302 MB > 256 MiB
    N, B = 6000, 4096
    rng = np.random.default_rng(7)
    key = np.unique(rng.integers(0, B, 3 * N) * N + np.repeat(np.arange(N), 3))
    big = G.Context(N, B, 0.001, precision="fp64")
    big.set_spikes((key // N).astype(np.int64), (key % N).astype(np.int32))
    big.set_kernel(0.01)
    st = lib.glmr_set_kernel_noalloc(big.handle, ctypes.c_double(0.02))
    assert st == G.L.GLMR_EINVAL and b"static scratch" in lib.glmr_last_error(big.handle)
    assert G.glmr_get_params(big.handle) == 0.01  # nothing changed
    big.close()
