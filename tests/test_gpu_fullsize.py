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


def test_full_size_fit_reaches_oracle_row_optima():
    """The headline reconstruction (BF16 ascent from J = 0 to its stopping
    test, then an FP32 polish from the BF16 optimum) against the oracle's exact
    optimum of sampled rows of the same recording (per-row Newton on the
    Hessian of Eq. (18), stored by tests/golden/make_config2_newton.py with the
    entries' standard errors).  Distances are in standard errors, the
    resolution the data allow.  Classes: the fit's k-means centroids (Sec. 3.3)
    applied to the oracle's rows give the fit's classes except for entries
    that the fit's own error could carry across a class boundary."""
    import json
    import os
    import paper_1502_04993_amd as G
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config2_newton_rows.json")))
    rec = synth.cached("config2", seed=0, B=3_600_000)
    fp = _fingerprint(rec)
    assert (fp["n_spikes"], fp["checksum"]) == (ref["recording"]["n_spikes"], ref["recording"]["checksum"])
    N, B = rec.n_neurons, rec.n_bins
    ctx = G.Context(N, B, rec.dt, precision="bf16")
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    rb = ctx.fit(max_iter=400, from_zero=True)
    Jb, mub, _ = ctx.get_params()
    ctx.set_precision("fp32")
    rp = ctx.fit(max_iter=60)
    Jp, mup, _ = ctx.get_params()
    ctx.close()
    print(f"[full fit] bf16 {rb}\n[full fit] fp32 polish {rp}", flush=True)
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
    print(f"[full fit] max |J - J_oracle| / SE: BF16 {zb:.3f}, after the FP32 polish {zp:.4f}; "
          f"mu {zmu:.4f}; class differences {flips} (all within the fit's error of a boundary: {near})",
          flush=True)
    # BF16 evaluates the likelihood at bf16(J) with a stochastically rounded
    # trace (gradient error ~3e-4): its optimum lies within the data's own
    # resolution, one standard error, of the exact one (0.14 measured on these
    # rows with the default history of 40, 0.50 with 10); the FP32 polish
    # brings it to a small fraction of it (0.0007)
    assert rb["converged"] and zb < 1.0
    assert zp < 0.05 and zmu < 0.05


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
