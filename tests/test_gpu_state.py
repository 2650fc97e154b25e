"""Checkpoint and resume of a fit (glmr_get_state, glmr_set_state,
fit(resume=True)) on the GPU (needs an MI355X).

Every reduction of the evaluation and of the ascent runs in a fixed order, so
the ascent is deterministic: a fit of a + b steps must equal, bit for bit, a
fit of a steps resumed for b steps, both in the same context and in a fresh
context of the same recording that restored the checkpoint.  The penalty and
bounds travel with the checkpoint.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _G():
    import paper_1502_04993_amd as G
    return G


def _ctx(rec, prec, tau=None):
    c = _G().Context(rec.n_neurons, rec.n_bins, rec.dt, precision=prec)
    c.set_spikes(rec.bins, rec.neurons)
    if tau is not None:
        c.set_kernel(tau)
    return c


@pytest.mark.parametrize("prec,pen", [("fp64", {}), ("fp64", dict(l1_alpha=2.0, j_max=1.5)),
                                      ("bf16", {})])
def test_resumed_fit_equals_uninterrupted(prec, pen):
    rec = synth.balanced(N=60, B=20_000, in_frac=0.3, seed=171)
    a, b = 6, 10
    full = _ctx(rec, prec, rec.tau)
    rf = full.fit(max_iter=a + b, from_zero=True, **pen)
    Jf, muf, _ = full.get_params()
    full.close()
    assert rf["iters"] == a + b and not rf["converged"]  # the cap, not the stopping test, ends it

    part = _ctx(rec, prec, rec.tau)
    r1 = part.fit(max_iter=a, from_zero=True, **pen)
    assert r1["iters"] == a and not r1["converged"]
    state = part.get_state()
    r2 = part.fit(max_iter=b, resume=True)
    Jp, mup, _ = part.get_params()
    part.close()
    print(f"[state {prec} {pen}] {len(state)} bytes; ll full {rf['ll']!r} resumed {r2['ll']!r}", flush=True)
    assert r2["iters"] == b and r2["evals"] == b  # no fresh start: one evaluation per step
    assert np.array_equal(Jp, Jf) and np.array_equal(mup, muf) and r2["ll"] == rf["ll"]

    # a fresh context of the same configuration, at another tau: the
    # checkpoint brings back its own, and the fit ends bit for bit where the
    # uninterrupted one did
    fresh = _ctx(rec, prec, 2.0 * rec.tau)
    fresh.set_state(state)
    assert fresh.get_params()[2] == rec.tau
    r3 = fresh.fit(max_iter=b, resume=True)
    Jr, mur, _ = fresh.get_params()
    fresh.close()
    assert np.array_equal(Jr, Jf) and np.array_equal(mur, muf) and r3["ll"] == rf["ll"]
    # a context created in another precision takes the checkpoint's; its
    # neuron padding (chosen at creation) may differ, which changes the
    # grouping of the sums.  In FP64 the path stays within rounding of the
    # uninterrupted one; in BF16 ten mid-ascent line searches on gradients
    # with 1e-4 noise may take other steps, so only the ascent's progress is
    # compared there
    other = "fp32" if prec != "fp32" else "fp64"
    alt = _ctx(rec, other, 2.0 * rec.tau)
    alt.set_state(state)
    assert alt.precision == prec
    r4 = alt.fit(max_iter=b, resume=True)
    Ja, _, _ = alt.get_params()
    alt.close()
    print(f"[state {prec} {pen}] other padding: ll {r4['ll']!r}, max|dJ| {np.abs(Ja - Jf).max():.3e}", flush=True)
    if prec == "fp64":
        assert np.abs(Ja - Jf).max() <= 1e-10 * np.abs(Jf).max()
    assert r4["ll"] > r1["ll"] and abs(r4["ll"] - rf["ll"]) <= 1e-3 * abs(rf["ll"])


def test_resume_to_convergence_and_parameters_only_checkpoint():
    rec = synth.balanced(N=40, B=20_000, in_frac=0.3, seed=172)
    c = _ctx(rec, "fp64", rec.tau)
    r1 = c.fit(max_iter=10, from_zero=True)
    r2 = c.fit(max_iter=2000, resume=True)
    assert r2["converged"] and r2["rows_converged"] == 40
    ref = _ctx(rec, "fp64", rec.tau)
    rr = ref.fit(max_iter=2000, from_zero=True)
    assert r1["iters"] + r2["iters"] == rr["iters"]
    assert np.array_equal(c.get_params()[0], ref.get_params()[0])
    # a converged ascent resumes to nothing
    r3 = c.fit(max_iter=50, resume=True)
    assert r3["iters"] == 0 and r3["converged"]
    # after set_params the ascent is gone: the checkpoint holds parameters only
    J, mu, _ = ref.get_params()
    ref.set_params(J, mu)
    s_par = ref.get_state()
    s_full = c.get_state()
    assert len(s_par) < len(s_full)
    ref.close()
    d = _ctx(rec, "fp64")
    d.set_state(s_par)
    assert np.array_equal(d.get_params()[0], J)
    with pytest.raises(_G().GlmrError) as e:
        d.fit(max_iter=5, resume=True)
    assert e.value.status == _G().L.GLMR_ESTATE
    d.close()
    c.close()


def test_checkpoint_rejections():
    G = _G()
    rec = synth.balanced(N=30, B=10_000, in_frac=0.3, seed=173)
    c = _ctx(rec, "fp64", rec.tau)
    with pytest.raises(G.GlmrError) as e:  # no parameters yet
        c.get_state()
    assert e.value.status == G.L.GLMR_ESTATE
    with pytest.raises(G.GlmrError) as e:  # nothing to resume
        c.fit(max_iter=5, resume=True)
    assert e.value.status == G.L.GLMR_ESTATE
    c.fit(max_iter=5, from_zero=True)
    st = c.get_state()
    # a changed kernel ends the ascent
    c.set_kernel(1.5 * rec.tau)
    with pytest.raises(G.GlmrError):
        c.fit(max_iter=5, resume=True)
    c.set_state(st)  # the checkpoint's tau and ascent come back
    assert c.get_params()[2] == rec.tau
    c.fit(max_iter=5, resume=True)
    # another recording (other spikes), another shape, damaged buffers
    rec2 = synth.balanced(N=30, B=10_000, in_frac=0.3, seed=174)
    o = _ctx(rec2, "fp64", rec.tau)
    bad = [st[:-8], st + b"\0" * 8, b"XXXXXXXX" + st[8:], st[:40]]
    for s in bad:
        with pytest.raises(G.GlmrError) as e:
            c.set_state(s)
        assert e.value.status == G.L.GLMR_EINVAL
    with pytest.raises(G.GlmrError) as e:
        o.set_state(st)
    assert e.value.status == G.L.GLMR_EINVAL
    # the same spikes at other times (the bins permuted): equal total and
    # per-neuron counts, another raster
    perm = np.random.default_rng(5).permutation(rec.n_bins)
    moved = _G().Context(rec.n_neurons, rec.n_bins, rec.dt, precision="fp64")
    moved.set_spikes(perm[rec.bins].astype(np.int64), rec.neurons)
    moved.set_kernel(rec.tau)
    with pytest.raises(G.GlmrError) as e:
        moved.set_state(st)
    assert e.value.status == G.L.GLMR_EINVAL and "raster" in str(e.value)
    moved.close()
    small = synth.balanced(N=20, B=10_000, in_frac=0.3, seed=173)
    s2 = _ctx(small, "fp64", rec.tau)
    with pytest.raises(G.GlmrError) as e:
        s2.set_state(st)
    assert e.value.status == G.L.GLMR_EINVAL
    # a batch fit starts afresh
    o.set_params(np.zeros((30, 30)), np.zeros(30))
    b = G.Batch([o])
    with pytest.raises(G.GlmrError):
        b.fit(max_iter=3, resume=True)
    b.close()
    for x in (c, o, s2):
        x.close()


def test_event_grid_fit_resumes_bit_for_bit():
    # the continuous-time model: the checkpoint keeps the time mode and the
    # event grid's slots; a context of the same events resumes the ascent
    G = _G()
    rec = synth.balanced(N=30, B=20_000, in_frac=0.3, seed=175)
    times, neu = synth.event_times(rec, seed=3)

    def ctx():
        c = G.Context.from_events(30, times, neu, 0.0, rec.T, precision="fp64")
        c.set_kernel(rec.tau)
        return c
    full = ctx()
    rf = full.fit(max_iter=16, from_zero=True)
    Jf = full.get_params()[0]
    full.close()
    part = ctx()
    part.fit(max_iter=6, from_zero=True)
    st = part.get_state()
    part.close()
    fresh = ctx()
    fresh.set_state(st)
    r = fresh.fit(max_iter=10, resume=True)
    Jr = fresh.get_params()[0]
    fresh.close()
    assert r["iters"] == 10 and np.array_equal(Jr, Jf) and r["ll"] == rf["ll"]
    # a regular-grid context of the same size refuses the checkpoint
    grid = G.Context(30, 20_000, rec.dt, precision="fp64")
    grid.set_spikes(rec.bins, rec.neurons)
    with pytest.raises(G.GlmrError) as e:
        grid.set_state(st)
    assert e.value.status == G.L.GLMR_EINVAL
    grid.close()
