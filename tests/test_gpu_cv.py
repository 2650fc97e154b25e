"""Cross-validation scans over tau and the l1 penalty (Sec. 2.5, Sec. 3.2),
GPU against the oracle (needs an MI355X).

The recording is split in time; every grid point is fitted on the first half
and scored by L(full) - L(training prefix) at the fitted parameters.  Without
the penalty the oracle fits the same prefix by exact Newton and scores it
with its own likelihood.  With the penalty the optimum is unique (strictly
concave objective), so the GPU's fitted parameters are checked against the
optimality conditions computed by the oracle, and its validation scores
against the oracle's scores of the same parameters.
"""
import numpy as np
import pytest

import synth
from oracle import glm_oracle as O

pytestmark = pytest.mark.gpu

TAUS = [0.004, 0.008, 0.016, 0.032]
ALPHA, EPS = 2.0, 1e-4
# the fit must shrink the gradient of the penalised objective to this
# fraction of its largest entry at the uncoupled start (J = 0, mu_i = log q_i/T)
GREL = 1e-3


def test_cv_scan_matches_oracle_and_finds_tau():
    from paper_1502_04993_amd.cv import cv_scan
    rec = synth.balanced(N=20, B=60_000, in_frac=0.25, tau=0.008, seed=13)
    N, B, dt = rec.n_neurons, rec.n_bins, rec.dt
    res = cv_scan(rec.bins, rec.neurons, N, B, dt, TAUS, alphas=[0.0, ALPHA], train_frac=0.5,
                  precision="fp32", max_iter=3000, l1_eps=EPS)
    print(f"[cv] gpu scan done, validation L {np.array2string(res.val, precision=3)}", flush=True)
    bt = res.train_bins
    assert bt == B // 2
    m = rec.bins < bt
    tb, tn = rec.bins[m], rec.neurons[m]

    def score(tau, J, mu):
        full = O.loglik(rec.bins, rec.neurons, N, B, dt, tau, J, mu)
        head = O.loglik(tb, tn, N, bt, dt, tau, J, mu)
        return full["ll_rows"] - head["ll_rows"], full["ll"], head

    ref = np.zeros(len(TAUS))
    for ti, tau in enumerate(TAUS):
        # no penalty: the oracle's own maximum likelihood fit of the prefix
        J, mu, _ = O.newton_fit(tb, tn, N, bt, dt, tau)
        v, _, _ = score(tau, J, mu)
        ref[ti] = v.sum()
        print(f"[cv] alpha=0 tau={tau}: gpu {res.val[0, ti]:.6f} oracle {ref[ti]:.6f}", flush=True)
        assert abs(res.val[0, ti] - ref[ti]) <= 1e-6 * abs(ref[ti])
        # penalised: score the GPU's parameters and check they maximise the
        # penalised training objective (its gradient vanishes there)
        Jg, mug = res.params[(1, ti)]
        vg, lfull, head = score(tau, Jg, mug)
        assert np.allclose(res.val_rows[1, ti], vg, rtol=0, atol=1e-9 * abs(lfull))
        _, dpen = O.l1_eps_penalty(Jg, ALPHA, EPS)
        gJ, gmu = head["gJ"] - dpen, head["gmu"]
        nz = np.abs(Jg) > 1e-2
        q = np.bincount(tn, minlength=N)
        g0 = O.loglik(tb, tn, N, bt, dt, tau, np.zeros((N, N)), np.log(q / (bt * dt)))["gJ"]
        gtol = GREL * np.abs(g0).max()
        print(f"[cv] alpha={ALPHA} tau={tau}: |J|>0.01 for {nz.sum()} of {N * N}, "
              f"max|grad J| {np.abs(gJ).max():.2e} max|grad mu| {np.abs(gmu).max():.2e} "
              f"report {res.reports[(1, ti)]}", flush=True)
        assert 0 < nz.sum() < N * N - N
        assert np.abs(gJ).max() <= gtol and np.abs(gmu).max() <= gtol
        if tau == 0.008:
            # the oracle's own penalised optimum of the prefix
            Jo, muo, _ = O.penalized_fit(tb, tn, N, bt, dt, tau, alpha=ALPHA, eps=EPS)
            vo, _, _ = score(tau, Jo, muo)
            print(f"[cv] alpha={ALPHA} tau={tau}: gpu {res.val[1, ti]:.6f} oracle {vo.sum():.6f} "
                  f"max|J-Jo| {np.abs(Jg - Jo).max():.2e}", flush=True)
            assert abs(res.val[1, ti] - vo.sum()) <= 1e-6 * abs(vo.sum())
            assert np.abs(Jg - Jo).max() <= 5e-3 and np.abs(mug - muo).max() <= 1e-3
    assert int(np.argmax(ref)) == TAUS.index(0.008)
    assert int(np.argmax(res.val[0])) == TAUS.index(0.008)
    a, t = res.best()
    assert res.val[res.alphas.index(a), res.taus.index(t)] == res.val.max()
    assert 0.004 <= res.mean_row_peak_tau(0) <= 0.016


def test_cv_scan_over_delays_scores_like_oracle_and_finds_no_delay():
    """Delay axis of the scan (Sec. 2.4, Fig. 4): the data carry no
    transmission delay beyond the grid's one bin, so d = 0 validates best; the
    GPU's validation scores equal the oracle's scores of the same parameters,
    and each fit is a stationary point of the oracle's delayed likelihood."""
    from paper_1502_04993_amd.cv import cv_scan
    rec = synth.balanced(N=20, B=60_000, in_frac=0.25, tau=0.008, seed=13)
    N, B, dt = rec.n_neurons, rec.n_bins, rec.dt
    delays = [(0, 0), (2, 0), (5, 1)]
    res = cv_scan(rec.bins, rec.neurons, N, B, dt, [0.008], precision="fp64", max_iter=3000,
                  delays=delays)
    bt = res.train_bins
    m = rec.bins < bt
    tb, tn = rec.bins[m], rec.neurons[m]
    for k, (d, ds) in enumerate(delays):
        J, mu = res.params[(0, k)]
        full = O.loglik_delayed(rec.bins, rec.neurons, N, B, dt, 0.008, J, mu, d, ds)
        head = O.loglik_delayed(tb, tn, N, bt, dt, 0.008, J, mu, d, ds)
        v = full["ll_rows"] - head["ll_rows"]
        g = max(np.abs(head["gJ"]).max(), np.abs(head["gmu"]).max())
        print(f"[cv delays] d={d} ds={ds}: gpu {res.val[0, k]:.6f} oracle {v.sum():.6f} max|grad| {g:.2e}",
              flush=True)
        assert np.allclose(res.val_rows[0, k], v, rtol=0, atol=1e-9 * abs(full["ll"]))
        assert g <= 1e-4
    assert res.best() == (0.0, 0.008, (0, 0))
