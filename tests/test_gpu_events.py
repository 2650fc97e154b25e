"""Continuous-time likelihood on the event grid (Sec. 2.3, Eq. (7)-(8), (10),
(12), (14)), GPU against the FP64 oracle (needs an MI355X).

Inputs: the synthetic rasters with every spike placed uniformly inside its
bin (continuous times, network events every ~1 ms).  Each comparison asserts
the total L, the largest per-row error of L_i, and the gradient error as a
2-norm and element-wise (tests/parity_check.py).  Bounds as for the regular
grid (the same arithmetic per slot; the interval integrals are FP64 in both
modes):
  FP64: L 1e-12, L_i 1e-11, gradient 1e-10
  FP32: L 1e-10 sqrt(2e6 / (slots N)) (stochastically rounded FP32 trace),
        L_i sqrt(N) times that, gradient 1e-6 (both contractions accumulate
        in FP64; measured 4e-9 - 6e-9).
  BF16: L 1e-3, L_i 1e-3, gradient 1e-3 (trace, J and the weights in BF16, the interval
        integrals from the FP32-accumulated potential).  "bf16" runs the
        resident BF16 trace (kernel U takes the integrals in its epilogue),
        "bf16-rc" the kernels that rebuild the trace from the spike masks.
"""
import math

import numpy as np
import pytest

import synth
from oracle import glm_oracle as O
from parity_check import check

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(ll=1e-12, row=1e-11, grad=1e-10, gmax=1e-10),
       "fp32": dict(ll=1e-10, row=1e-10, grad=1e-6, gmax=1e-6),
       "bf16": dict(ll=1e-3, row=1e-3, grad=1e-3, gmax=1e-3),
       "bf16-rc": dict(ll=1e-3, row=1e-3, grad=1e-3, gmax=1e-3)}


def _G():
    import paper_1502_04993_amd as G
    return G


def _lists(times, neurons, N):
    return [times[neurons == j] for j in range(N)]


def _ctx(N, times, neurons, T0, T1, prec, max_gap=0.0, chunk_bins=0, allow_silent=False):
    G = _G()
    slots = G.glmr_event_slots(times, T0, T1, max_gap)
    trace = "recompute" if prec.endswith("-rc") else "auto"
    c = G.Context(N, slots, (T1 - T0) / slots, prec.split("-")[0], chunk_bins=chunk_bins,
                  time_mode="events", trace=trace)
    try:
        c.set_spike_times(times, neurons, T0, T1, max_gap)
    except G.GlmrError as e:
        if not (allow_silent and e.status == G.L.GLMR_ENOSPIKES):
            raise
    return c, slots


def _compare(r, ref, prec, slots, N, label, q=None):
    tol = dict(TOL[prec])
    if prec == "fp32":
        tol["ll"] *= max(1.0, (2e6 / (slots * N)) ** 0.5)
        tol["row"] = 4.0 * tol["ll"] * N ** 0.5
    if q is not None:  # the integral term of each row, dL/dmu_i = q_i - integral
        ref = dict(ref, integral_term=np.asarray(q, float) - ref["gmu"])
    check(f"events {label} {prec} slots={slots}", r, ref, tol)


def _round(J, prec):
    if prec.startswith("bf16"):
        import torch
        return torch.tensor(J).to(torch.bfloat16).to(torch.float64).numpy()
    return J.astype(np.float32).astype(np.float64) if prec == "fp32" else J


@pytest.mark.parametrize("prec,N,B,chunk", [("fp64", 70, 30_000, 0), ("fp32", 70, 30_000, 0),
                                            ("bf16", 70, 30_000, 0),
                                            ("fp64", 150, 12_000, 4096), ("fp32", 150, 12_000, 4096),
                                            ("bf16", 150, 12_000, 4096), ("bf16", 300, 8_000, 0),
                                            ("bf16", 400, 6_000, 0), ("bf16-rc", 70, 30_000, 0),
                                            ("bf16-rc", 150, 12_000, 4096), ("bf16-rc", 400, 6_000, 0)])
def test_event_grid_matches_oracle(prec, N, B, chunk):
    # N = 150 pads to two neuron tiles; chunk_bins = 4096 splits the slots
    # into several chunks with a ragged last one; BF16 at N = 400 runs the
    # 256-neuron tiles (the others 128)
    rec = synth.balanced(N=N, B=B, in_frac=0.3, seed=91 + N)
    times, neu = synth.event_times(rec, seed=5)
    T0, T1 = 0.0, rec.T
    c, slots = _ctx(N, times, neu, T0, T1, prec, chunk_bins=chunk)
    c.set_kernel(rec.tau)
    J = _round(rec.J, prec)
    c.set_params(J, rec.mu)
    r = c.eval(grad=True)
    resident = c.query()["trace_resident"]
    c.close()
    assert resident == (prec == "bf16")
    ref = O.continuous_eval(_lists(times, neu, N), T0, T1, rec.tau, J, rec.mu)
    _compare(r, ref, prec, slots, N, f"N={N} q={times.shape[0]} chunk={chunk}", q=np.bincount(neu, minlength=N))


@pytest.mark.parametrize("prec", ["bf16", "bf16-rc"])
def test_event_grid_rare_tiers_and_mixed_slots(prec):
    # a sparse, strongly coupled network (2 spikes/s per neuron, couplings
    # 2.5x the default): about 60 % of the (slot, neuron) intervals lie past
    # the FP32 expansion's bound (the quadrature and FP64 tiers), and in about
    # 30 % of the slots some neurons' intervals are past it and others not,
    # so the BF16 kernels' per-slot branch takes mixed slots (counted on the
    # host from the events, as in the oracle's recursion of Eq. (8)).  BF16
    # only: the FP32 chain of the interval integrals is the BF16 modes' (FP64
    # and FP32 take the FP64 evaluation)
    N = 70
    rec = synth.balanced(N=N, B=30_000, in_frac=0.3, j_exc=0.5, j_inh=-1.5, rate_lo=1.0, rate_hi=3.0,
                         seed=177)
    times, neu = synth.event_times(rec, seed=5)
    T0, T1 = 0.0, rec.T
    c, slots = _ctx(N, times, neu, T0, T1, prec)
    c.set_kernel(rec.tau)
    J = _round(rec.J, prec)
    c.set_params(J, rec.mu)
    r = c.eval(grad=True)
    c.close()
    o = np.lexsort((neu, times))
    ts, ns = np.concatenate([times[o], [T1]]), neu[o]
    v, t_prev, past, mixed = np.zeros(N), T0, 0, 0
    for m in range(ts.shape[0]):
        delta = (ts[m] - t_prev) / rec.tau
        if m >= 1:
            v[ns[m - 1]] += 1.0
        out = delta * np.maximum(1.0, np.abs((J @ v) * np.exp(-delta / 2))) > 0.35
        past += int(out.sum())
        mixed += int(out.any() and not out.all())
        v *= np.exp(-delta)
        t_prev = ts[m]
    assert past > 0.3 * N * ts.shape[0] and mixed > 0.1 * ts.shape[0], (past, mixed)
    ref = O.continuous_eval(_lists(times, neu, N), T0, T1, rec.tau, J, rec.mu)
    _compare(r, ref, prec, slots, N, "rare tiers", q=np.bincount(neu, minlength=N))


def test_event_grid_without_events_is_poisson():
    G = _G()
    N, T0, T1 = 3, 0.5, 2.5
    c, slots = _ctx(N, np.zeros(0), np.zeros(0, np.int32), T0, T1, "fp64", allow_silent=True)
    c.set_kernel(0.01)
    mu = np.log(np.array([2.0, 5.0, 0.5]))
    c.set_params(np.array([[0.3, -1.0, 0.0], [2.0, 0.1, 0.4], [0.0, 0.0, -3.0]]), mu)
    r = c.eval(grad=True)
    c.close()
    assert slots == 1  # default max_gap 4 (T1 - T0): the window is one slot
    assert np.allclose(r["ll_rows"], -np.exp(mu) * (T1 - T0), rtol=1e-13)
    assert np.allclose(r["gmu"], -np.exp(mu) * (T1 - T0), rtol=1e-13)
    assert np.all(r["gJ"] == 0.0)
    assert G is not None


def test_event_grid_ties_first_event_and_long_gaps():
    # an event at T0, equal times of different neurons, and a silent stretch
    # of 2 s that max_gap = 0.05 s splits into spike-free slots
    rng = np.random.default_rng(3)
    N, T0, T1, tau = 5, 0.0, 6.0, 0.02
    ts = [np.sort(np.concatenate([rng.random(12), 3.0 + 3.0 * rng.random(14)])) for _ in range(N)]
    ts[0] = np.sort(np.concatenate([[0.0, 0.5, 3.5], ts[0]]))
    ts[2] = np.sort(np.concatenate([[0.5, 3.5], ts[2]]))
    ts[4] = np.sort(np.concatenate([[3.5], ts[4]]))
    times = np.concatenate(ts)
    neu = np.concatenate([np.full(t.shape[0], j, np.int32) for j, t in enumerate(ts)])
    order = np.lexsort((neu, times))
    times, neu = times[order], neu[order]
    J = rng.normal(0, 0.8, (N, N))
    mu = np.log(rng.uniform(3, 8, N))
    ref = O.continuous_eval(ts, T0, T1, tau, J, mu)
    out = []
    for mg in (0.0, 0.05):
        c, slots = _ctx(N, times, neu, T0, T1, "fp64", max_gap=mg)
        c.set_kernel(tau)
        c.set_params(J, mu)
        r = c.eval(grad=True)
        c.close()
        _compare(r, ref, "fp64", slots, N, f"ties max_gap={mg}")
        out.append((slots, r))
    assert out[1][0] > out[0][0] + 40  # the silent 2 s alone takes 40 slots at 0.05 s
    # splitting intervals leaves the likelihood unchanged
    assert abs(out[0][1]["ll"] - out[1][1]["ll"]) <= 1e-12 * abs(out[0][1]["ll"])


def test_event_grid_rejections():
    G = _G()
    rec = synth.balanced(N=20, B=5_000, seed=7)
    times, neu = synth.event_times(rec, seed=1)
    c, _ = _ctx(20, times, neu, 0.0, rec.T, "fp64")
    # events out of (time, neuron) order, out of the window, or a slot count
    # that does not match the context
    with pytest.raises(G.GlmrError):
        c.set_spike_times(times[::-1].copy(), neu[::-1].copy(), 0.0, rec.T)
    with pytest.raises(G.GlmrError):
        c.set_spike_times(times, neu, 0.0, times[-1])
    with pytest.raises(G.GlmrError):
        c.set_spike_times(times, neu, 0.0, rec.T, max_gap=1e-4)
    with pytest.raises(G.GlmrError):
        c.set_spikes(rec.bins, rec.neurons)
    c.set_spike_times(times, neu, 0.0, rec.T)
    c.set_kernel(rec.tau)
    c.set_params(rec.J, rec.mu)
    with pytest.raises(G.GlmrError):
        c.eval(want_tau=True)
    with pytest.raises(G.GlmrError):
        c.set_precision("fp8")
    c.close()
    # a run of 64 slots longer than 600 tau is refused when the tables are built
    sparse = np.array([0.0, 50.0, 100.0])
    sn = np.array([0, 1, 0], np.int32)
    c2, _ = _ctx(2, sparse, sn, 0.0, 200.0, "fp64", max_gap=1e9)
    with pytest.raises(G.GlmrError):
        c2.set_kernel(1e-3)
    c2.set_kernel(1.0)  # 200 s span = 200 tau: fine
    c2.close()


def test_event_grid_fit_reaches_oracle_optimum():
    rec = synth.balanced(N=20, B=40_000, in_frac=0.3, seed=17)
    times, neu = synth.event_times(rec, seed=2)
    N, T0, T1 = 20, 0.0, rec.T
    c, slots = _ctx(N, times, neu, T0, T1, "fp64")
    c.set_kernel(rec.tau)
    rep = c.fit(max_iter=2000, from_zero=True)
    J, mu, _ = c.get_params()
    c.close()
    lists = _lists(times, neu, N)
    ref = O.continuous_eval(lists, T0, T1, rec.tau, J, mu)
    q = np.bincount(neu, minlength=N)
    g0 = O.continuous_eval(lists, T0, T1, rec.tau, np.zeros((N, N)), np.log(q / (T1 - T0)))
    gmax0 = np.abs(g0["gJ"]).max()
    gmax = max(np.abs(ref["gJ"]).max(), np.abs(ref["gmu"]).max())
    print(f"[events fit] {rep} slots={slots} max|grad| {gmax:.3e} (start {gmax0:.3e}) "
          f"ll gpu {rep['ll']:.10f} oracle {ref['ll']:.10f}", flush=True)
    assert rep["rows_converged"] == N
    assert gmax <= 1e-5 * gmax0
    assert abs(rep["ll"] - ref["ll"]) <= 1e-12 * abs(ref["ll"])
    # the fitted couplings recover the simulated ones' signs where they are strong
    strong = np.abs(rec.J) >= 0.5
    np.fill_diagonal(strong, False)
    assert np.mean(np.sign(J[strong]) == np.sign(rec.J[strong])) > 0.8


def test_event_grid_bf16_tile_shapes_and_autotune(tmp_path):
    # kernel U's event-grid variants: the fragment-major kernel (shape 7, the
    # default) with kernel G's fragment tiles 7, 8, 9, 10, and the row-major
    # 128-neuron tiles (shapes 3-6, GLMR_XFRAG=0); every one matches the
    # oracle, they agree with each other far inside the tolerance, and the
    # autotuner keeps the event grid's choice apart from the regular grid's in
    # a shared cache
    import os
    G = _G()
    N = 512
    rec = synth.balanced(N=N, B=5_000, in_frac=0.3, seed=93)
    times, neu = synth.event_times(rec, seed=6)
    T0, T1 = 0.0, rec.T
    J = _round(rec.J, "bf16")
    ref = O.continuous_eval(_lists(times, neu, N), T0, T1, rec.tau, J, rec.mu)
    lls = []
    for u, g, frag in [(7, 7, True), (7, 8, True), (7, 9, True), (7, 10, True), (3, 2, False), (4, 2, False), (5, 2, False),
                       (6, 2, False)]:
        os.environ["GLMR_RES_SHAPE"] = f"{u},{g}"
        if not frag:
            os.environ["GLMR_XFRAG"] = "0"
        try:
            c, slots = _ctx(N, times, neu, T0, T1, "bf16")
        finally:
            os.environ.pop("GLMR_RES_SHAPE", None)
            os.environ.pop("GLMR_XFRAG", None)
        c.set_kernel(rec.tau)
        c.set_params(J, rec.mu)
        r = c.eval(grad=True)
        assert c.query()["trace_resident"] and c.query()["trace_frag"] == frag
        c.close()
        _compare(r, ref, "bf16", slots, N, f"shape {u},{g}")
        lls.append(r["ll"])
    assert max(abs(v - lls[0]) for v in lls) <= 1e-9 * abs(lls[0])
    cache = str(tmp_path / "tune.txt")
    c, _ = _ctx(N, times, neu, T0, T1, "bf16")
    c.set_kernel(rec.tau)
    c.set_params(J, rec.mu)
    u, g = c.autotune(cache)
    c.close()
    assert u == 7 and g in (7, 8, 9, 10)
    grid = G.Context(N, rec.n_bins, rec.dt, "bf16")
    grid.set_spikes(rec.bins, rec.neurons)
    grid.set_kernel(rec.tau)
    grid.set_params(J, rec.mu)
    grid.autotune(cache)
    grid.close()
    lines = open(cache).read().splitlines()
    print(f"[events autotune] u={u} g={g}; cache {lines}", flush=True)
    assert len(lines) == 2 and lines[0].split()[1:5] != lines[1].split()[1:5]
