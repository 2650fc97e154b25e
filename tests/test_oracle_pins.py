"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a brute-force
sum, a closed form, a quadrature, finite differences, an invariant, or a value
printed in the paper.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import glm_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def tiny_raster(N=4, B=300, rate=0.04, seed=0, multi=True):
    rng = np.random.default_rng(seed)
    S = (rng.random((B, N)) < rate).astype(np.int64)
    if multi:
        S[rng.integers(0, B, 3), rng.integers(0, N, 3)] += 1  # a few bins with 2+ spikes
    bins, neu = [], []
    for t in range(B):
        for i in range(N):
            for _ in range(S[t, i]):
                bins.append(t)
                neu.append(i)
    return np.array(bins, np.int64), np.array(neu, np.int32), S.astype(np.float64)


# --------------------------------------------------------------- trace (P-a)

def test_trace_three_ways():
    bins, neu, S = tiny_raster()
    a = O.decay(0.001, 0.004)
    Xr = O.trace_recursive(S, a)
    Xd = O.trace_direct(S, a)
    Xl = O.trace_lfilter(S, a)
    assert np.allclose(Xr, Xd, rtol=1e-14, atol=1e-15)
    assert np.allclose(Xl, Xd, rtol=1e-14, atol=1e-15)
    # causality: a spike in bin t' does not act on bin t'; first weight is 1
    S1 = np.zeros((10, 1)); S1[3, 0] = 1
    X1 = O.trace_direct(S1, a)
    assert X1[3, 0] == 0.0 and X1[4, 0] == 1.0 and abs(X1[6, 0] - a * a) < 1e-16


def test_trace_carry_and_chunking():
    bins, neu, S = tiny_raster(B=500, seed=3)
    a = O.decay(0.001, 0.01)
    X = O.trace_lfilter(S, a)
    # restart the filter at row 137 from the carried value
    x0 = a * X[136] + S[136]
    X2 = O.trace_lfilter(S[137:], a, x0)
    assert np.allclose(X2, X[137:], rtol=1e-13, atol=1e-15)
    N, B = S.shape[1], S.shape[0]
    J = np.random.default_rng(1).normal(0, 0.3, (N, N))
    mu = np.log(np.array([5.0, 7.0, 9.0, 6.0]))
    r1 = O.loglik(bins, neu, N, B, 0.001, 0.01, J, mu, want_tau=True, chunk=7)
    r2 = O.loglik(bins, neu, N, B, 0.001, 0.01, J, mu, want_tau=True, chunk=100000)
    assert abs(r1["ll"] - r2["ll"]) <= 1e-13 * abs(r2["ll"])
    assert np.allclose(r1["gJ"], r2["gJ"], rtol=1e-12, atol=1e-12)
    assert abs(r1["gtau"] - r2["gtau"]) <= 1e-10 * abs(r2["gtau"])


def test_tau_trace_matches_direct_and_fd():
    bins, neu, S = tiny_raster(B=200, seed=5)
    dt, tau = 0.001, 0.006
    a = O.decay(dt, tau)
    X, Y = O.tau_trace_recursive(S, a, dt, tau)
    Yd = O.tau_trace_direct(S, a, dt, tau)
    assert np.allclose(Y, Yd, rtol=1e-13, atol=1e-15)
    h = 1e-7
    Xp = O.trace_direct(S, O.decay(dt, tau + h))
    Xm = O.trace_direct(S, O.decay(dt, tau - h))
    assert np.allclose((Xp - Xm) / (2 * h), Y, rtol=1e-6, atol=1e-6)


# -------------------------------------------------- closed forms at J = 0 (P-b)

def test_closed_form_at_zero_coupling():
    bins, neu, S = tiny_raster(N=5, B=400, seed=7)
    N, B = 5, 400
    dt, tau = 0.001, 0.008
    a = O.decay(dt, tau)
    mu = np.log(np.array([3.0, 5.0, 8.0, 11.0, 2.0]))
    r = O.loglik(bins, neu, N, B, dt, tau, np.zeros((N, N)), mu)
    q = np.bincount(neu, minlength=N)
    T = B * dt
    # U = mu everywhere: L_i = q_i mu_i - T e^{mu_i}
    assert np.allclose(r["ll_rows"], q * mu - T * np.exp(mu), rtol=1e-13)
    assert np.allclose(r["gmu"], q - T * np.exp(mu), rtol=1e-12, atol=1e-12)
    # gradient from spike times only (pairwise sums over spike lists)
    times = [bins[neu == j] for j in range(N)]
    for i in range(N):
        for j in range(N):
            dsig = sum(a ** (t - tp - 1) for t in times[i] for tp in times[j] if tp < t)
            integ = math.exp(mu[i]) * dt * sum((1 - a ** (B - 1 - tp)) / (1 - a) for tp in times[j])
            assert abs(r["gJ"][i, j] - (dsig - integ)) <= 1e-11 * (1 + abs(dsig))


def test_spike_term_identity():
    """Sum_t s_i U_i = q_i mu_i + sum_j J_ij dSigma_ij (U is linear in theta)."""
    bins, neu, S = tiny_raster(N=6, B=500, seed=11)
    N, B = 6, 500
    rng = np.random.default_rng(2)
    J = rng.normal(0, 0.5, (N, N))
    mu = rng.normal(1.5, 0.2, N)
    r = O.loglik(bins, neu, N, B, 0.001, 0.01, J, mu)
    D = O.spike_term_matrix(bins, neu, N, B, 0.001, 0.01)
    q = np.bincount(neu, minlength=N)
    assert np.allclose(r["spike_term"], q * mu + (J * D).sum(axis=1), rtol=1e-13)
    # dSigma is the spike-time sum of the trace (independent of J, mu)
    X = O.trace_direct(S, O.decay(0.001, 0.01))
    assert np.allclose(D, S.T @ X, rtol=1e-13)


# ----------------------------------------------------- uncoupled MLE (P-c)

def test_uncoupled_mle_closed_form():
    bins, neu, S = tiny_raster(N=4, B=2000, rate=0.01, seed=13, multi=False)
    N, B, dt = 4, 2000, 0.001
    J, mu, info = O.newton_fit(bins, neu, N, B, dt, 0.01, fit_J=False)
    q = np.bincount(neu, minlength=N)
    assert np.allclose(np.exp(mu), q / (B * dt), rtol=1e-13)


# ----------------------------------- continuous time, quadrature (P-d)

def _times(N=3, T=1.0, rate=12.0, seed=0):
    rng = np.random.default_rng(seed)
    return [np.sort(rng.random(rng.poisson(rate * T)) * T) for _ in range(N)]


def test_ei_closed_form_matches_quadrature():
    ts = _times(seed=1)
    J = np.array([[-1.0, 0.6, -0.4], [0.3, -2.0, 0.9], [0.0, -0.7, -1.2]])
    mu = np.log(np.array([6.0, 9.0, 4.0]))
    ei = O.continuous_ll(ts, 0.0, 1.0, 0.02, J, mu, method="ei")
    qd = O.continuous_ll(ts, 0.0, 1.0, 0.02, J, mu, method="quad")
    assert np.allclose(ei, qd, rtol=1e-11, atol=1e-11)


def test_eq14_matches_quadrature_and_fd():
    ts = _times(seed=2)
    J = np.array([[-1.0, 0.6, -0.4], [0.3, -2.0, 0.9], [0.0, -0.7, -1.2]])
    mu = np.log(np.array([6.0, 9.0, 4.0]))
    tau = 0.02
    for i in range(3):
        cf = O.continuous_grad_integral(ts, 0.0, 1.0, tau, J, mu, i, method="closed")
        qd = O.continuous_grad_integral(ts, 0.0, 1.0, tau, J, mu, i, method="quad")
        assert np.allclose(cf, qd, rtol=1e-10, atol=1e-12)
        # Eq. (12): dL_i/dJ_ij = sum_k v_ij(t_ik) - integral; check by FD of Eq. (10)
        h = 1e-6
        for j in range(3):
            Jp = J.copy(); Jp[i, j] += h
            Jm = J.copy(); Jm[i, j] -= h
            fd = (O.continuous_ll(ts, 0, 1, tau, Jp, mu)[i] - O.continuous_ll(ts, 0, 1, tau, Jm, mu)[i]) / (2 * h)
            vsum = sum(math.exp(-(t - tp) / tau) for t in ts[i] for tp in ts[j] if tp < t)
            assert abs(fd - (vsum - cf[j])) < 1e-6 * (1 + abs(fd))


def test_ei_small_argument_branch():
    # Ei(D) - Ei(D xi) for tiny D: series branch vs direct with a moderate D
    for D in (1e-3, -1e-3, 5e-3):
        xi = 0.7
        import scipy.special as sp
        direct = sp.expi(D) - sp.expi(D * xi)
        assert abs(O._ei_diff(D, xi) - direct) < 1e-11


def test_continuous_eval_matches_event_loops_and_fd():
    ts = _times(N=3, seed=5)
    J = np.array([[-1.0, 0.6, -0.4], [0.3, -2.0, 0.9], [0.0, -0.7, -1.2]])
    mu = np.log(np.array([6.0, 9.0, 4.0]))
    tau = 0.02
    r = O.continuous_eval(ts, 0.0, 1.0, tau, J, mu)
    # the row-by-row loops of Eq. (8)/(10), themselves pinned by quadrature
    assert np.allclose(r["ll_rows"], O.continuous_ll(ts, 0.0, 1.0, tau, J, mu), rtol=1e-12, atol=1e-12)
    for i in range(3):
        gi = O.continuous_grad_integral(ts, 0.0, 1.0, tau, J, mu, i)
        vsum = np.array([sum(math.exp(-(t - tp) / tau) for t in ts[i] for tp in ts[j] if tp < t)
                         for j in range(3)])
        assert np.allclose(r["gJ"][i], vsum - gi, rtol=1e-11, atol=1e-11)
    # gradient against central differences of the row likelihoods
    h = 1e-6
    for i in range(3):
        mp, mm = mu.copy(), mu.copy()
        mp[i] += h
        mm[i] -= h
        fd = (O.continuous_ll(ts, 0, 1, tau, J, mp)[i] - O.continuous_ll(ts, 0, 1, tau, J, mm)[i]) / (2 * h)
        assert abs(fd - r["gmu"][i]) < 1e-6 * (1 + abs(fd))
        for j in range(3):
            Jp, Jm = J.copy(), J.copy()
            Jp[i, j] += h
            Jm[i, j] -= h
            fd = (O.continuous_ll(ts, 0, 1, tau, Jp, mu)[i] - O.continuous_ll(ts, 0, 1, tau, Jm, mu)[i]) / (2 * h)
            assert abs(fd - r["gJ"][i, j]) < 1e-6 * (1 + abs(fd))


def test_continuous_eval_without_events_is_poisson():
    # no spikes: U_i = mu_i throughout, L_i = -e^{mu_i} (T1 - T0)
    mu = np.log(np.array([2.0, 5.0]))
    J = np.array([[0.3, -1.0], [2.0, 0.1]])
    r = O.continuous_eval([np.array([]), np.array([])], 1.5, 4.0, 0.01, J, mu)
    assert np.allclose(r["ll_rows"], -np.exp(mu) * 2.5, rtol=1e-14)
    assert np.allclose(r["gmu"], -np.exp(mu) * 2.5, rtol=1e-14)
    assert np.all(r["gJ"] == 0.0)


def test_continuous_eval_equal_times_are_the_limit_of_ordered_times():
    # two events at the same time act in (time, neuron) order: the same as the
    # limit of neuron 1 firing just after neuron 0
    J = np.array([[-0.5, 0.8], [1.2, -0.3]])
    mu = np.log(np.array([4.0, 3.0]))
    tie = O.continuous_eval([np.array([0.2, 0.5]), np.array([0.5, 0.7])], 0.0, 1.0, 0.03, J, mu)
    near = O.continuous_eval([np.array([0.2, 0.5]), np.array([0.5 + 1e-10, 0.7])], 0.0, 1.0, 0.03, J, mu)
    assert np.allclose(tie["ll_rows"], near["ll_rows"], rtol=0, atol=1e-7)
    assert np.allclose(tie["gJ"], near["gJ"], rtol=0, atol=1e-7)


def test_grid_converges_to_continuous_first_order():
    ts = _times(N=3, T=2.0, rate=8.0, seed=4)
    J = np.array([[-1.0, 0.6, -0.4], [0.3, -2.0, 0.9], [0.0, -0.7, -1.2]])
    mu = np.log(np.array([6.0, 9.0, 4.0]))
    tau = 0.02
    exact = O.continuous_ll(ts, 0.0, 2.0, tau, J, mu)
    errs = []
    for dt in (1e-3, 5e-4, 2.5e-4, 1.25e-4):
        g = O.grid_ll_from_times(ts, 2.0, dt, tau, J, mu)
        errs.append(np.abs(g - exact).sum())
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    # O(dt): halving dt halves the error
    assert all(1.6 < r < 2.5 for r in ratios), (errs, ratios)
    assert errs[-1] < 0.05 * np.abs(exact).sum()


# ------------------------------------------------------- concavity (P-e)

def test_concavity_hessian_and_monotone_gradient():
    bins, neu, S = tiny_raster(N=4, B=600, seed=17)
    N, B, dt, tau = 4, 600, 0.001, 0.01
    rng = np.random.default_rng(5)
    def grad(J, mu):
        r = O.loglik(bins, neu, N, B, dt, tau, J, mu)
        return np.concatenate([r["gmu"], r["gJ"].ravel()])
    def ll(J, mu):
        return O.loglik(bins, neu, N, B, dt, tau, J, mu, want_grad=False)["ll"]
    J0 = rng.normal(0, 0.5, (N, N)); mu0 = rng.normal(2, 0.3, N)
    # Hessian by FD of the analytic gradient, per row block (separable)
    P = N + N * N
    theta0 = np.concatenate([mu0, J0.ravel()])
    H = np.zeros((P, P))
    h = 1e-5
    for k in range(P):
        tp = theta0.copy(); tp[k] += h
        tm = theta0.copy(); tm[k] -= h
        H[:, k] = (grad(tp[N:].reshape(N, N), tp[:N]) - grad(tm[N:].reshape(N, N), tm[:N])) / (2 * h)
    H = 0.5 * (H + H.T)
    assert np.linalg.eigvalsh(H).max() <= 1e-6 * np.abs(H).max()
    for _ in range(5):
        d = rng.normal(size=P); d /= np.linalg.norm(d)
        e = 1e-3
        f = lambda t: ll((theta0 + t * d)[N:].reshape(N, N), (theta0 + t * d)[:N])
        assert f(e) + f(-e) - 2 * f(0) <= 1e-9
        t1 = theta0 + 0.3 * d
        g0 = grad(J0, mu0); g1 = grad(t1[N:].reshape(N, N), t1[:N])
        assert float((g1 - g0) @ (t1 - theta0)) <= 0.0


# ------------------------------------------- finite differences (P-f)

def test_gradient_finite_differences_including_tau():
    bins, neu, S = tiny_raster(N=4, B=500, seed=19)
    N, B, dt, tau = 4, 500, 0.001, 0.009
    rng = np.random.default_rng(9)
    J = rng.normal(0, 0.5, (N, N)); mu = rng.normal(2, 0.3, N)
    r = O.loglik(bins, neu, N, B, dt, tau, J, mu, want_tau=True)
    h = 1e-6
    for i in range(N):
        for j in range(N):
            Jp = J.copy(); Jp[i, j] += h
            Jm = J.copy(); Jm[i, j] -= h
            fp = O.loglik(bins, neu, N, B, dt, tau, Jp, mu, want_grad=False)["ll_rows"][i]
            fm = O.loglik(bins, neu, N, B, dt, tau, Jm, mu, want_grad=False)["ll_rows"][i]
            assert abs((fp - fm) / (2 * h) - r["gJ"][i, j]) < 1e-6 * (1 + abs(r["gJ"][i, j]))
        mp = mu.copy(); mp[i] += h
        mm = mu.copy(); mm[i] -= h
        fd = (O.loglik(bins, neu, N, B, dt, tau, J, mp, want_grad=False)["ll_rows"][i]
              - O.loglik(bins, neu, N, B, dt, tau, J, mm, want_grad=False)["ll_rows"][i]) / (2 * h)
        assert abs(fd - r["gmu"][i]) < 1e-6 * (1 + abs(fd))
    ht = 1e-7
    fd = (O.loglik(bins, neu, N, B, dt, tau + ht, J, mu, want_grad=False)["ll"]
          - O.loglik(bins, neu, N, B, dt, tau - ht, J, mu, want_grad=False)["ll"]) / (2 * ht)
    assert abs(fd - r["gtau"]) < 1e-5 * (1 + abs(fd))


# ------------------------------------------------------ separability (P-i)

def test_separability():
    bins, neu, S = tiny_raster(N=5, B=400, seed=23)
    N, B = 5, 400
    rng = np.random.default_rng(3)
    J = rng.normal(0, 0.5, (N, N)); mu = rng.normal(2, 0.3, N)
    r1 = O.loglik(bins, neu, N, B, 0.001, 0.01, J, mu)
    J2 = J.copy(); J2[1:] = rng.normal(0, 0.5, (N - 1, N)); mu2 = mu.copy(); mu2[1:] += 0.3
    r2 = O.loglik(bins, neu, N, B, 0.001, 0.01, J2, mu2)
    assert r1["ll_rows"][0] == r2["ll_rows"][0]
    assert np.array_equal(r1["gJ"][0], r2["gJ"][0]) and r1["gmu"][0] == r2["gmu"][0]


# --------------------------------------------------------- fits (P-g)

def test_newton_fit_reaches_optimum():
    import synth
    rec = synth.erdos_renyi(N=12, B=6000, p=0.3, seed=2)
    N, B = rec.n_neurons, rec.n_bins
    J, mu, info = O.newton_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau)
    r0 = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, np.zeros((N, N)), np.zeros(N))
    r = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu)
    g0 = np.concatenate([r0["gmu"], r0["gJ"].ravel()])
    g = np.concatenate([r["gmu"], r["gJ"].ravel()])
    assert np.linalg.norm(g) <= 1e-8 * np.linalg.norm(g0)
    # at the optimum the expected spike count equals the observed one (Sec. 2.3.3)
    assert np.allclose(r["integral_term"], r["q"], rtol=1e-9)
    # L-BFGS-B on the joint vector converges to the same optimum
    J2, mu2, res = O.lbfgs_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau)
    assert np.allclose(J2, J, atol=2e-4) and np.allclose(mu2, mu, atol=2e-4)


# ------------------------------------------------- metrics (P-j) and k-means

def test_mer0_printed_values():
    gold = json.load(open(GOLDEN))
    for row in gold["mer0"]:
        v = 100.0 * O.mer0(row["p"], row["f_e"])
        assert round(v, 2) == row["mer0_percent"]
        assert abs(O.mer0_counts(row["p"], row["f_e"], 1000) - O.mer0(row["p"], row["f_e"])) < 1e-15


def test_mer0_monte_carlo():
    """A random classifier that keeps p, f_e, f_i misclassifies MER_0 of the pairs."""
    rng = np.random.default_rng(0)
    N, p, fe = 400, 0.2, 0.8
    n_exc = int(fe * N)
    vals = []
    for trial in range(5):
        conn = rng.random((N, N)) < p
        Jt = np.where(conn, np.where(np.arange(N)[None, :] < n_exc, 1.0, -1.0), 0.0)
        np.fill_diagonal(Jt, 0)
        conn2 = rng.random((N, N)) < p
        exc2 = rng.random((N, N)) < fe
        labels = np.where(conn2, np.where(exc2, 2, 0), 1)
        np.fill_diagonal(labels, -1)
        vals.append(O.mer(labels, Jt)["mer"])
    assert abs(np.mean(vals) - O.mer0(p, fe)) < 0.003


def test_confusion_bookkeeping_matches_tables():
    """Rebuild label sets with the error counts of Tables 2 and 6: each error
    sits in two rows, so the total is half the row sum over N^2."""
    gold = json.load(open(GOLDEN))
    for tab in gold["confusion_tables"]:
        N = tab["N"]
        rows = tab["rows"]
        n_err = rows["excitatory"]["errors"]
        n_fp = int(round(n_err * rows["excitatory"]["fp_percent"] / 100))
        n_fn = n_err - n_fp
        Jt = np.zeros((N, N))
        # excitatory truth on the first block of pairs
        idx = np.argwhere(~np.eye(N, dtype=bool))
        Jt[idx[: 50_000, 0], idx[: 50_000, 1]] = 0.5
        labels = np.where(Jt > 0, 2, 1)
        np.fill_diagonal(labels, -1)
        fn_pairs = idx[:n_fn]                  # true E, labelled none
        fp_pairs = idx[50_000:50_000 + n_fp]   # true none, labelled E
        labels[fn_pairs[:, 0], fn_pairs[:, 1]] = 1
        labels[fp_pairs[:, 0], fp_pairs[:, 1]] = 2
        m = O.mer(labels, Jt)
        assert m["rows"]["excitatory"]["errors"] == rows["excitatory"]["errors"]
        assert m["rows"]["unconnected"]["errors"] == rows["unconnected"]["errors"]
        assert m["rows"]["inhibitory"]["errors"] == 0
        assert m["half_row_sum"] == m["errors"]
        assert round(100 * m["mer_n2"], 2) == tab["total_percent"]


def test_kmeans3_fixed_point():
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.normal(-1, 0.05, 200), rng.normal(0, 0.05, 2000), rng.normal(0.2, 0.05, 300)])
    lab, c = O.kmeans3(v)
    assert c[0] < c[1] < c[2]
    # fixed point: each value is nearest to its own centroid, each centroid is its cluster mean
    assert np.array_equal(lab, np.argmin(np.abs(v[:, None] - c[None, :]), axis=1))
    for k in range(3):
        assert abs(c[k] - v[lab == k].mean()) < 1e-12
    assert (lab[:200] == 0).all()


def test_row_subset_is_the_same_definition():
    bins, neu, S = tiny_raster(N=6, B=700, seed=29)
    N, B = 6, 700
    rng = np.random.default_rng(4)
    J = rng.normal(0, 0.5, (N, N)); mu = rng.normal(2, 0.3, N)
    full = O.loglik(bins, neu, N, B, 0.001, 0.01, J, mu, want_tau=True)
    sub = O.loglik(bins, neu, N, B, 0.001, 0.01, J, mu, want_tau=True, rows=[4, 1])
    assert np.array_equal(sub["ll_rows"], full["ll_rows"][[4, 1]])
    assert np.allclose(sub["gJ"], full["gJ"][[4, 1]], rtol=1e-13, atol=1e-13)
    assert np.array_equal(sub["gmu"], full["gmu"][[4, 1]])


def test_validation_likelihood_is_full_minus_training_prefix():
    """The trace is causal, so the log-likelihood of the bins after a split,
    with the whole recording as history, is the full L minus the L of the
    training prefix alone (the identity the cross-validation scans use)."""
    import synth
    rec = synth.balanced(N=15, B=8000, in_frac=0.3, seed=4)
    N, B = rec.n_neurons, rec.n_bins
    rng = np.random.default_rng(5)
    J = rec.J + rng.normal(0, 0.05, (N, N))
    bt = 4700
    full = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, rec.mu)
    tail = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, rec.mu, bin_range=(bt, B))
    m = rec.bins < bt
    head = O.loglik(rec.bins[m], rec.neurons[m], N, bt, rec.dt, rec.tau, J, rec.mu)
    assert np.allclose(full["ll_rows"] - head["ll_rows"], tail["ll_rows"], rtol=1e-12, atol=1e-9)


# ---------------------------------------------------- delays (Sec. 2.4, Eq. (15))

def _delayed_row_by_shifted_raster(S, i, d, ds, a, dt, J, mu):
    """Eq. (15) literally for row i: shift every spike train S_j by its delay
    (d, or d_self for j = i), filter the shifted raster, and take the spike
    terms at the recorded spikes of i."""
    B, N = S.shape
    Sh = np.zeros_like(S)
    for j in range(N):
        D = ds if j == i else d
        if D < B:
            Sh[D:, j] = S[:B - D, j]
    X = O.trace_recursive(Sh, a)
    U = mu[i] + X @ J[i]
    return float((S[:, i] * U).sum() - dt * np.exp(U).sum())


@pytest.mark.parametrize("d,ds", [(0, 0), (3, 1), (2, 2), (0, 4), (70, 1)])
def test_delayed_likelihood_is_eq15_row_by_row(d, ds):
    bins, neu, S = tiny_raster(N=5, B=700, seed=21)
    N, B, dt, tau = 5, 700, 0.001, 0.01
    rng = np.random.default_rng(2)
    J = rng.normal(0, 0.6, (N, N))
    mu = rng.normal(3.0, 0.3, N)
    r = O.loglik_delayed(bins, neu, N, B, dt, tau, J, mu, d, ds)
    for i in range(N):
        ref = _delayed_row_by_shifted_raster(S, i, d, ds, O.decay(dt, tau), dt, J, mu)
        assert abs(r["ll_rows"][i] - ref) <= 1e-11 * abs(ref)
    if d == ds == 0:
        u = O.loglik(bins, neu, N, B, dt, tau, J, mu)
        assert np.allclose(r["ll_rows"], u["ll_rows"], rtol=1e-13)
        assert np.allclose(r["gJ"], u["gJ"], rtol=1e-12, atol=1e-12)


def test_delayed_gradient_matches_finite_differences():
    bins, neu, S = tiny_raster(N=4, B=600, seed=22)
    N, B, dt, tau, d, ds = 4, 600, 0.001, 0.01, 3, 1
    rng = np.random.default_rng(4)
    J = rng.normal(0, 0.6, (N, N))
    mu = rng.normal(3.0, 0.3, N)
    r = O.loglik_delayed(bins, neu, N, B, dt, tau, J, mu, d, ds)
    h = 1e-6
    for (i, j) in [(0, 1), (2, 2), (3, 0), (1, 1)]:
        Jp, Jm = J.copy(), J.copy()
        Jp[i, j] += h
        Jm[i, j] -= h
        fd = (O.loglik_delayed(bins, neu, N, B, dt, tau, Jp, mu, d, ds)["ll_rows"][i]
              - O.loglik_delayed(bins, neu, N, B, dt, tau, Jm, mu, d, ds)["ll_rows"][i]) / (2 * h)
        assert abs(fd - r["gJ"][i, j]) < 1e-6 * (1 + abs(fd))
    mp, mm = mu.copy(), mu.copy()
    mp[2] += h
    mm[2] -= h
    fd = (O.loglik_delayed(bins, neu, N, B, dt, tau, J, mp, d, ds)["ll_rows"][2]
          - O.loglik_delayed(bins, neu, N, B, dt, tau, J, mm, d, ds)["ll_rows"][2]) / (2 * h)
    assert abs(fd - r["gmu"][2]) < 1e-6 * (1 + abs(fd))


def test_newton_rows_chunked_matches_dense_newton_and_kkt():
    """The oracle's chunked per-row Newton (the full-size reference fits) reaches
    the dense per-row Newton's optimum with chunk boundaries inside the
    recording (2e4 bins in chunks of 3000: a ragged last chunk), and the
    likelihood's own gradient vanishes there (App. A: a concave row problem
    has one maximiser)."""
    import synth
    rec = synth.config1(0)
    N, B = rec.n_neurons, rec.n_bins
    rows = [0, 7, 45]
    res = O.newton_rows(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, rows, chunk=3000)
    # the trace rebuilt on every pass instead of kept: the same iterates
    res2 = O.newton_rows(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, rows, chunk=3000, cache_bytes=0)
    for i in rows:
        assert np.array_equal(res[i]["J"], res2[i]["J"]) and res[i]["iters"] == res2[i]["iters"]
    Jn, mun, _ = O.newton_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, rows=rows)
    J = np.zeros((N, N))
    mu = np.zeros(N)
    for i in rows:
        assert np.abs(res[i]["J"] - Jn[i]).max() < 1e-8 and abs(res[i]["mu"] - mun[i]) < 1e-9
        J[i], mu[i] = res[i]["J"], res[i]["mu"]
    r = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu, rows=rows)
    q = O.spike_counts(rec.neurons, N)
    r0 = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, np.zeros((N, N)), np.log(q / (B * rec.dt)),
                  rows=rows)
    for k, i in enumerate(rows):
        assert res[i]["ll"] == pytest.approx(float(r["ll_rows"][k]), rel=1e-13)
        g = np.abs(np.concatenate([[r["gmu"][k]], r["gJ"][k]])).max()
        g0 = np.abs(np.concatenate([[r0["gmu"][k]], r0["gJ"][k]])).max()
        assert g <= 1e-9 * g0


def test_newton_rows_sub_reaches_dense_newton_optimum_and_kkt():
    """The subsampled-Newton-matrix row fit (the many-row full-size reference)
    reaches the dense per-row Newton's optimum: its steps use a Hessian of
    Eq. (18) taken on every second chunk only, but it iterates on the exact
    gradient, whose zero is the one maximiser of the concave row problem
    (App. A).  Chunks of 3000 bins leave a ragged last chunk; the rows are
    given out of order."""
    import synth
    rec = synth.config1(0)
    N, B = rec.n_neurons, rec.n_bins
    rows = [45, 0, 7, 23]
    res = O.newton_rows_sub(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, rows, hess_stride=2,
                            refresh=2, chunk=3000)
    Jn, mun, _ = O.newton_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, rows=rows)
    J = np.zeros((N, N))
    mu = np.zeros(N)
    for i in rows:
        assert np.abs(res[i]["J"] - Jn[i]).max() < 1e-8 and abs(res[i]["mu"] - mun[i]) < 1e-9
        J[i], mu[i] = res[i]["J"], res[i]["mu"]
    r = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu, rows=rows)
    q = O.spike_counts(rec.neurons, N)
    r0 = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, np.zeros((N, N)), np.log(q / (B * rec.dt)),
                  rows=rows)
    for k, i in enumerate(rows):
        assert res[i]["ll"] == pytest.approx(float(r["ll_rows"][k]), rel=1e-13)
        g = np.abs(np.concatenate([[r["gmu"][k]], r["gJ"][k]])).max()
        g0 = np.abs(np.concatenate([[r0["gmu"][k]], r0["gJ"][k]])).max()
        assert g <= 1e-9 * g0
        assert res[i]["max_abs_grad"] == pytest.approx(g, rel=1e-3, abs=1e-12 * g0)
        # the standard-error estimate is positive and finite
        assert np.all(np.isfinite(res[i]["se"])) and np.all(res[i]["se"] > 0)


@pytest.mark.parametrize("chunk", [7, 50, 65536])
def test_continuous_eval_rows_is_the_all_rows_evaluator(chunk):
    """The rows-restricted continuous evaluator (for event lists too long for
    the all-rows loop) gives continuous_eval's rows: L_i, dL/dJ_i. and dL/dmu_i
    of Eq. (7), (10), (12), (14), with chunk boundaries anywhere, an event at
    T0, equal times of different neurons, and rows out of order."""
    rng = np.random.default_rng(17)
    N, T0, T1, tau = 6, 0.0, 2.0, 0.015
    ts = [np.sort(rng.random(int(rng.integers(8, 20))) * (T1 - T0) + T0) for _ in range(N)]
    ts[0] = np.sort(np.concatenate([[T0], ts[0]]))
    ts[3] = np.sort(np.concatenate([ts[3], [ts[1][2]]]))  # a tie with neuron 1
    J = rng.normal(0.0, 0.8, (N, N))
    J[2] = 0.0  # D = 0 throughout for this row
    J[4, :] *= 1e-4  # |D| in the series branch
    mu = np.log(rng.uniform(3.0, 9.0, N))
    ref = O.continuous_eval(ts, T0, T1, tau, J, mu)
    times = np.concatenate(ts)
    neu = np.concatenate([np.full(len(t), j) for j, t in enumerate(ts)]).astype(np.int32)
    order = np.lexsort((neu, times))
    rows = [5, 0, 2, 4, 3, 1]
    r = O.continuous_eval_rows(times[order], neu[order], N, T0, T1, tau, J, mu, rows, chunk=chunk)
    assert np.allclose(r["ll_rows"], ref["ll_rows"][rows], rtol=1e-12, atol=1e-12)
    assert np.allclose(r["gJ"], ref["gJ"][rows], rtol=1e-11, atol=1e-11)
    assert np.allclose(r["gmu"], ref["gmu"][rows], rtol=1e-12, atol=1e-12)
    assert np.array_equal(r["q"], np.array([len(ts[i]) for i in rows], dtype=float))
    sub = O.continuous_eval_rows(times[order], neu[order], N, T0, T1, tau, J, mu, [3], chunk=chunk)
    assert np.allclose(sub["ll_rows"], ref["ll_rows"][[3]], rtol=1e-12, atol=1e-12)
