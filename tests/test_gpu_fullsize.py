"""Parity at the headline size (N = 1000, 3.6e6 bins, 23.8 M spikes), in the
launch configuration the bench times (resident trace, default chunking, the
autotuned tile shapes), on sampled rows that the FP64 oracle evaluates over
the whole recording: L is separable over rows (Sec. 2.2), so L_i, dL/dmu_i and
the full row dL/dJ_i. of a few neurons are exact references at any N.

L_i and the gradient rows are compared at the simulated parameters and at
theta = 0.  At the simulated parameters of a 3.6e6-bin recording the gradient
is nearly zero (they are close to the maximum), a small difference of the
spike term and the lambda term, which makes it the sensitive point: an FP32
accumulation of the lambda term over long time splits (~1e-5 of the term)
showed there as a 9e-4 error, hence the FP64 accumulation of kernel G.
Needs an MI355X; about a minute and a half of host time for the oracle.
"""
import numpy as np
import pytest

import synth
from oracle import glm_oracle as O
from parity_check import check
from test_gpu_parity import round_fp8_rows

pytestmark = pytest.mark.gpu

ROWS = [0, 257, 799, 800, 999]  # first and last excitatory, first and last inhibitory, one inside
# Per-row L_i (the FP32 target 1e-10: at 3.6e6 bins a row averages as many
# terms as the whole likelihood of the small parity cases), and the gradient
# rows as a 2-norm and element-wise (tests/parity_check.py); the same bounds as
# the parity tests.
TOL = {"fp32": dict(row=1e-10, grad=1e-6, gmax=1e-6),
       "bf16": dict(row=1e-3, grad=1e-3, gmax=1e-3),
       "fp8": dict(row=5e-3, grad=3e-2, gmax=3e-2)}


def _bf16(J):
    import torch
    return torch.tensor(J).to(torch.bfloat16).to(torch.float64).numpy()


def test_full_size_sampled_rows(tmp_path):
    import paper_1502_04993_amd as G
    rec = synth.cached("config2", seed=0, B=3_600_000)
    N, B = rec.n_neurons, rec.n_bins
    print(f"[full] recording ready: N={N} B={B} spikes={rec.n_spikes}", flush=True)
    Jb, J8 = _bf16(rec.J), round_fp8_rows(rec.J)
    Z = np.zeros((N, N))
    refs = {}
    for tag, J, mu in (("bf16", Jb, rec.mu), ("fp8", J8, rec.mu), ("zero", Z, np.zeros(N))):
        refs[tag] = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu, rows=ROWS)
        print(f"[full] oracle rows {ROWS} at {tag} done", flush=True)
    for prec in ("bf16", "fp8", "fp32"):
        J = J8 if prec == "fp8" else Jb  # BF16 values are exact in FP32
        ref = refs["fp8" if prec == "fp8" else "bf16"]
        ctx = G.Context(N, B, rec.dt, precision=prec)
        ctx.set_spikes(rec.bins, rec.neurons)
        ctx.set_kernel(rec.tau)
        if prec != "fp32":
            ctx.set_params(J, rec.mu)
            ctx.autotune(str(tmp_path / "tune.txt"))
        ctx.set_params(J, rec.mu)
        r = ctx.eval(grad=True)
        ctx.set_params(Z, np.zeros(N))
        r0 = ctx.eval(grad=True)
        q = ctx.query()
        ctx.close()
        assert q["trace_resident"] == (prec != "fp32")
        check(f"full {prec} at the simulated theta", r, ref, TOL[prec], rows=ROWS)
        check(f"full {prec} at theta = 0", r0, refs["zero"], TOL[prec], rows=ROWS)


def _fingerprint(rec):
    """Spike count and a checksum of the (bin, neuron) pairs (as the reference stores them)."""
    b = rec.bins.astype(np.int64)
    n = rec.neurons.astype(np.int64)
    return dict(n_spikes=int(b.shape[0]), checksum=int(np.sum((b * 1009 + n) % 1000003)))


_FITS = {}


def headline_fit(polish):
    """The headline reconstruction: BF16 ascent from J = 0 to its stopping
    test, then a continuation in `polish` ("fp32", or "bf16j2": BF16 with J in
    two BF16 terms) from the BF16 optimum.  Kept per polish for the tests of
    this module: (J_bf16, J, mu, reports, seconds)."""
    import time
    import paper_1502_04993_amd as G
    if polish not in _FITS:
        rec = synth.cached("config2", seed=0, B=3_600_000)
        N, B = rec.n_neurons, rec.n_bins
        ctx = G.Context(N, B, rec.dt, precision="bf16")
        ctx.set_spikes(rec.bins, rec.neurons)
        ctx.set_kernel(rec.tau)
        t0 = time.perf_counter()
        rb = ctx.fit(max_iter=400, from_zero=True)
        Jb, _, _ = ctx.get_params()
        t1 = time.perf_counter()
        ctx.set_precision(polish)
        rp = ctx.fit(max_iter=60 if polish == "fp32" else 400)
        t2 = time.perf_counter()
        Jp, mup, _ = ctx.get_params()
        ctx.close()
        print(f"[full fit] bf16 {rb} ({t1 - t0:.2f} s)\n[full fit] {polish} continuation {rp} "
              f"({t2 - t1:.2f} s)", flush=True)
        _FITS[polish] = (Jb, Jp, mup, (rb, rp), (t1 - t0, t2 - t1))
    return _FITS[polish]


# largest distance, in standard errors, of the continued fit from the oracle's
# exact row optima (measured: FP32 0.0007)
POLISH_Z = {"fp32": 0.05, "bf16j2": 0.05}


@pytest.mark.parametrize("polish", ["fp32", "bf16j2"])
def test_full_size_fit_reaches_oracle_row_optima(polish):
    """The headline reconstruction (BF16 ascent from J = 0 to its stopping
    test, then a continuation from the BF16 optimum in FP32 or in BF16 with a
    two-term J) against the oracle's exact optimum of sampled rows of the same
    recording (per-row Newton on the Hessian of Eq. (18), stored by
    tests/golden/make_config2_newton.py with the entries' standard errors).
    Distances are in standard errors, the resolution the data allow.
    Classes: the fit's k-means centroids (Sec. 3.3) applied to the oracle's
    rows give the fit's classes except for entries that the fit's own error
    could carry across a class boundary."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config2_newton_rows.json")))
    rec = synth.cached("config2", seed=0, B=3_600_000)
    fp = _fingerprint(rec)
    assert (fp["n_spikes"], fp["checksum"]) == (ref["recording"]["n_spikes"], ref["recording"]["checksum"])
    N = rec.n_neurons
    Jb, Jp, mup, (rb, rp), _ = headline_fit(polish)
    _, c = O.kmeans3(Jp[~np.eye(N, dtype=bool)])
    bounds = np.array([(c[0] + c[1]) / 2, (c[1] + c[2]) / 2])
    lab = O.classify(Jp)
    zb = zp = zmu = 0.0
    flips = near = 0
    for r in ref["rows"]:
        i = r["row"]
        Jr = np.array([float(v) for v in r["J"]])
        se = np.array(r["se_J"])
        zb = max(zb, float(np.max(np.abs(Jb[i] - Jr) / se)))
        zp = max(zp, float(np.max(np.abs(Jp[i] - Jr) / se)))
        zmu = max(zmu, abs(mup[i] - float(r["mu"])) / r["se_mu"])
        off = np.arange(N) != i
        lab_ref = np.argmin(np.abs(Jr[:, None] - c[None, :]), axis=1)
        close = np.min(np.abs(Jr[:, None] - bounds[None, :]), axis=1) <= 2 * np.abs(Jp[i] - Jr) + 1e-12
        differ = (lab[i] != lab_ref) & off
        flips += int(np.sum(differ))
        near += int(np.sum(differ & close))
        assert np.all(~differ | close), (i, np.nonzero(differ & ~close))
    print(f"[full fit] max |J - J_oracle| / SE: BF16 {zb:.3f}, after the {polish} continuation {zp:.4f}; "
          f"mu {zmu:.4f}; class differences {flips} (all within the fit's error of a boundary: {near})",
          flush=True)
    # BF16 evaluates the likelihood at bf16(J), whose steps (up to 0.0156 at
    # |J| ~ 5) reach 0.13 standard errors; its optimum lies within that
    # resolution of the exact one (0.14 measured).  FP32, or BF16 with J in two
    # terms (steps 2^-16 relative), remove that quantisation.
    assert rb["converged"] and zb < 1.0
    assert zp < POLISH_Z[polish] and zmu < POLISH_Z[polish]


def test_full_size_classification_matches_oracle_rows():
    """The classification of the headline reconstruction (the bench's recipe:
    BF16 ascent, then the two-term-J continuation) against the oracle's
    optimum of 65 rows stratified by type (tests/golden/config2_optimum_rows.json):
    the same host k-means (Sec. 3.3, App. C.2) on the off-diagonal entries of
    those rows of both fits gives the same labels, except entries within
    1e-3 of the spread of a decision boundary of either side (reading R16);
    that count is reported (expected 0).  Also the MER of each side against
    the generating weights on those rows (Eq. (20))."""
    ref = _golden("config2_optimum_rows.json")
    rec = synth.cached("config2", seed=0, B=3_600_000)
    fp = _fingerprint(rec)
    assert (fp["n_spikes"], fp["checksum"]) == (ref["recording"]["n_spikes"], ref["recording"]["checksum"])
    N = rec.n_neurons
    rows = [r["row"] for r in ref["rows"]]
    Jo = np.array([[float(v) for v in r["J"]] for r in ref["rows"]])
    _, Jp, _, _, secs = headline_fit("bf16j2")
    Jf = Jp[rows]
    off = np.ones(Jo.shape, dtype=bool)
    off[np.arange(len(rows)), rows] = False

    def labels(M):
        lab, cen = O.kmeans3(M[off])
        spread = M[off].max() - M[off].min()
        bnd = np.array([(cen[0] + cen[1]) / 2, (cen[1] + cen[2]) / 2])
        near = np.min(np.abs(M[off][:, None] - bnd[None, :]), axis=1) <= 1e-3 * spread
        return lab, near, cen

    lo, near_o, co = labels(Jo)
    lf, near_f, cf = labels(Jf)
    differ = lo != lf
    bad = differ & ~(near_o | near_f)
    truth = O.truth_classes(rec.J)[rows][off]
    mer_o = float(np.mean(lo != truth))
    mer_f = float(np.mean(lf != truth))
    print(f"[classification] {len(rows)} rows, {off.sum()} entries: labels differ at {int(differ.sum())} "
          f"(near a boundary: {int((differ & (near_o | near_f)).sum())}); centroids oracle {co} fit {cf}; "
          f"MER oracle {mer_o:.4%} fit {mer_f:.4%}; fit time {sum(secs):.2f} s", flush=True)
    assert not bad.any(), np.nonzero(bad)


def _golden(name):
    import json
    import os
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))


def _rows_ref(point):
    return dict(ll_rows=np.array([float(v) for v in point["ll_rows"]]),
                gmu=np.array([float(v) for v in point["gmu"]]),
                gJ=np.array([[float(v) for v in row] for row in point["gJ"]]))


EV_TOL = {"fp64": dict(row=1e-11, grad=1e-10, gmax=1e-10),
          "fp32": dict(row=1e-10, grad=1e-6, gmax=1e-6),
          "bf16": dict(row=1e-3, grad=1e-3, gmax=1e-3)}


@pytest.mark.parametrize("prec", ["bf16", "fp64", "fp32"])
def test_event_grid_full_size_rows(prec, tmp_path):
    """Continuous time at the headline size (23.8 M events, 24.3 M slots,
    N = 1000) in the bench's launch configuration (default chunking; BF16:
    resident trace, autotuned tiles), every index far past 2^31, against the
    oracle's continuous-time rows stored by tests/golden/make_events_full_rows.py
    (Eq. (7)-(8), (10), (12), (14)), at the BF16-rounded simulated weights and
    at theta = 0."""
    import paper_1502_04993_amd as G
    gold = _golden("events_config2_rows.json")
    rows = gold["rows"]
    rec = synth.cached("config2", seed=0, B=3_600_000)
    N = rec.n_neurons
    times, neu = synth.event_times(rec, seed=0)
    meta = gold["recording"]
    assert times.shape[0] == meta["n_events"] and int(np.sum(neu.astype(np.int64))) == meta["neuron_sum"]
    assert float(np.sum(times)) == float(meta["time_sum"])
    print(f"[events full {prec}] {times.shape[0]} events ready", flush=True)
    ctx = G.Context.from_events(N, times, neu, 0.0, rec.T, precision=prec)
    ctx.set_kernel(rec.tau)
    J = _bf16(rec.J)
    ctx.set_params(J, rec.mu)
    if prec == "bf16":
        ctx.autotune(str(tmp_path / "tune.txt"))
    r = ctx.eval(grad=True)
    ctx.set_params(np.zeros((N, N)), np.zeros(N))
    r0 = ctx.eval(grad=True)
    q = ctx.query()
    ctx.close()
    print(f"[events full {prec}] slots={q['b_pad']} chunk={q['chunk_bins']} resident={q['trace_resident']}",
          flush=True)
    assert q["trace_resident"] == (prec == "bf16")
    check(f"events full {prec} at the simulated theta", r, _rows_ref(gold["points"]["bf16"]), EV_TOL[prec],
          rows=rows)
    check(f"events full {prec} at theta = 0", r0, _rows_ref(gold["points"]["zero"]), EV_TOL[prec], rows=rows)
