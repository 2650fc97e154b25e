"""Transmission delays (Sec. 2.4, Eq. (15)) on the GPU against the FP64 oracle
(needs an MI355X).

d bins on every connection j -> i (j != i), d_s bins on the self-connection;
the spike terms stay at the recorded bins.  (d, d_s) = (70, 1) crosses a
64-bin subtile; (0, 4) has only the self-delay; (2, 2) is a uniform delay
(a pure shift of the trace, also in FP8).  Bounds as in the parity tests of
the undelayed model: the total L, every L_i, and the gradient as a 2-norm and
element-wise (tests/parity_check.py).
"""
import numpy as np
import pytest

import synth
from oracle import glm_oracle as O
from parity_check import check
from test_gpu_parity import round_fp8_rows, tol_for

pytestmark = pytest.mark.gpu

PAIRS = [(3, 1), (2, 2), (0, 4), (70, 1)]


def _G():
    import paper_1502_04993_amd as G
    return G


def _J(J, prec):
    p = prec.split("-")[0]
    if p == "fp32":
        return J.astype(np.float32).astype(np.float64)
    if p == "bf16":
        import torch
        return torch.tensor(J).to(torch.bfloat16).to(torch.float64).numpy()
    if p == "fp8":
        return round_fp8_rows(J)
    return J


def _ctx(rec, prec, chunk_bins=0):
    G = _G()
    p = prec.split("-")[0]
    trace = "recompute" if prec.endswith("-rc") else "auto"
    c = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision=p, chunk_bins=chunk_bins, trace=trace)
    c.set_spikes(rec.bins, rec.neurons)
    return c


def _check(r, ref, prec, rec, label):
    tol = tol_for(prec, rec)
    check(f"delays {label} {prec}", r, ref, tol)
    # the self-coupling column has its own delay: its error on its own scale
    dg = np.abs(np.diag(r["gJ"]) - np.diag(ref["gJ"])).max() / np.abs(np.diag(ref["gJ"])).max()
    print(f"[delays {label} {prec}] diag={dg:.3e}", flush=True)
    assert dg <= max(tol["grad"], 1e-12) * 10


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "bf16-rc", "fp8"])
@pytest.mark.parametrize("N,B,chunk", [(70, 30_000, 0), (150, 12_000, 4096)])
def test_delays_match_oracle(prec, N, B, chunk):
    rec = synth.balanced(N=N, B=B, in_frac=0.3, seed=130 + N)
    J = _J(rec.J, prec)
    c = _ctx(rec, prec, chunk)
    c.set_kernel(rec.tau)
    c.set_params(J, rec.mu)
    base = c.eval(grad=True)
    for d, ds in PAIRS:
        if prec == "fp8" and d != ds:
            with pytest.raises(_G().GlmrError):
                c.set_delays(d, ds)
            continue
        c.set_delays(d, ds)
        r = c.eval(grad=True)
        ref = O.loglik_delayed(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, rec.mu, d, ds)
        _check(r, ref, prec, rec, f"N={N} d={d} ds={ds}")
    # back to no delay: bitwise the undelayed evaluation
    c.set_delays(0, 0)
    r = c.eval(grad=True)
    assert r["ll"] == base["ll"] and np.array_equal(r["gJ"], base["gJ"])
    c.close()


def test_delays_set_before_spikes_and_tau_gradient():
    G = _G()
    rec = synth.balanced(N=40, B=20_000, in_frac=0.3, seed=141)
    c = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision="fp64")
    c.set_delays(2, 2)  # before the spikes: applied at ingest
    c.set_spikes(rec.bins, rec.neurons)
    c.set_kernel(rec.tau)
    c.set_params(rec.J, rec.mu)
    r = c.eval(grad=True, want_tau=True)
    ref = O.loglik_delayed(rec.bins, rec.neurons, 40, rec.n_bins, rec.dt, rec.tau, rec.J, rec.mu, 2, 2)
    _check(r, ref, "fp64", rec, "before-spikes d=2 ds=2")
    # dL/dtau of the uniformly delayed model against central differences of L
    h = 1e-6 * rec.tau
    lp = lm = None
    for sgn in (1, -1):
        c.set_kernel(rec.tau + sgn * h)
        v = c.eval(grad=False)["ll"]
        lp, lm = (v, lm) if sgn == 1 else (lp, v)
    fd = (lp - lm) / (2 * h)
    print(f"[delays tau] grad {r['gtau']:.8e} fd {fd:.8e}", flush=True)
    assert abs(r["gtau"] - fd) <= 1e-5 * abs(fd)
    c.set_kernel(rec.tau)
    c.set_delays(3, 1)
    with pytest.raises(G.GlmrError):
        c.eval(want_tau=True)
    c.close()


def test_delayed_fit_reaches_oracle_optimum():
    rec = synth.balanced(N=20, B=40_000, in_frac=0.3, seed=151)
    N, B, d, ds = 20, 40_000, 2, 1
    c = _ctx(rec, "fp64")
    c.set_delays(d, ds)
    c.set_kernel(rec.tau)
    rep = c.fit(max_iter=2000, from_zero=True)
    J, mu, _ = c.get_params()
    c.close()
    ref = O.loglik_delayed(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu, d, ds)
    q = np.bincount(rec.neurons, minlength=N)
    g0 = O.loglik_delayed(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, np.zeros((N, N)),
                          np.log(q / (B * rec.dt)), d, ds)
    gmax = max(np.abs(ref["gJ"]).max(), np.abs(ref["gmu"]).max())
    print(f"[delays fit] {rep} max|grad| {gmax:.3e} (start {np.abs(g0['gJ']).max():.3e})", flush=True)
    assert rep["rows_converged"] == N
    assert gmax <= 1e-5 * np.abs(g0["gJ"]).max()
    assert abs(rep["ll"] - ref["ll"]) <= 1e-12 * abs(ref["ll"])


def test_batch_with_self_delay_equals_each_context():
    G = _G()
    recs = [synth.balanced(N=n, B=b, seed=160 + k) for k, (n, b) in enumerate([(70, 9_000), (130, 12_000)])]
    ctxs = []
    for k, r in enumerate(recs):
        c = _ctx(r, "bf16")
        c.set_delays(3, 1 if k == 0 else 3)
        c.set_kernel(r.tau)
        c.set_params(_J(r.J, "bf16"), r.mu)
        ctxs.append(c)
    singles = [c.eval(grad=True) for c in ctxs]
    b = G.Batch(ctxs)
    lls = b.eval()
    for k, c in enumerate(ctxs):
        gJ, gmu = b.grad(k)
        assert lls[k] == singles[k]["ll"] and np.array_equal(gJ, singles[k]["gJ"])
    b.close()
    for c in ctxs:
        c.close()
