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
from test_gpu_parity import round_fp8_rows

pytestmark = pytest.mark.gpu

ROWS = [0, 257, 799, 800, 999]  # first and last excitatory, first and last inhibitory, one inside
TOL = {"fp32": (1e-9, 1e-4), "bf16": (1e-3, 1e-3), "fp8": (2e-3, 3e-2)}


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
        rl = np.abs(r["ll_rows"][ROWS] - ref["ll_rows"]) / np.abs(ref["ll_rows"])
        gt = np.concatenate([r["gmu"][ROWS], r["gJ"][ROWS].ravel()])
        gtr = np.concatenate([ref["gmu"], ref["gJ"].ravel()])
        rgt = np.linalg.norm(gt - gtr) / np.linalg.norm(gtr)
        z = refs["zero"]
        g = np.concatenate([r0["gmu"][ROWS], r0["gJ"][ROWS].ravel()])
        gr = np.concatenate([z["gmu"], z["gJ"].ravel()])
        rg = np.linalg.norm(g - gr) / np.linalg.norm(gr)
        rl0 = np.abs(r0["ll_rows"][ROWS] - z["ll_rows"]) / np.abs(z["ll_rows"])
        print(f"[full {prec}] max rel L_i {rl.max():.3e} (theta = 0: {rl0.max():.3e}), rel grad rows "
              f"{rgt:.3e} (theta = 0: {rg:.3e})", flush=True)
        assert rl.max() <= TOL[prec][0] and rl0.max() <= TOL[prec][0]
        assert rgt <= TOL[prec][1] and rg <= TOL[prec][1]


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
