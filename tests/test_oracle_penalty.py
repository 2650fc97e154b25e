"""Pins of the oracle's penalised, bound-constrained fit (Sec. 2.5, 2.6.3:
the smooth epsilon-l1 penalty of Eq. (16)-(17), bounds on J and on the base
rates), against limits and optimality conditions that do not depend on how
the fit is computed."""
import math

import numpy as np
import pytest

import synth
from oracle import glm_oracle as O


def tiny():
    return synth.balanced(N=10, B=30000, in_frac=0.3, seed=3)


def test_penalty_limits_and_derivative():
    rng = np.random.default_rng(1)
    J = rng.normal(0, 0.7, (6, 6))
    # eps -> 0: alpha times the l1 norm of the off-diagonal weights of each row
    pen, _ = O.l1_eps_penalty(J, 0.3, 1e-30)
    off = J.copy()
    np.fill_diagonal(off, 0.0)
    assert np.allclose(pen, 0.3 * np.abs(off).sum(axis=1), rtol=1e-12)
    # the self-connection is not penalised
    J2 = J.copy()
    np.fill_diagonal(J2, 100.0)
    assert np.allclose(O.l1_eps_penalty(J2, 0.3, 1e-4)[0], O.l1_eps_penalty(J, 0.3, 1e-4)[0], rtol=0)
    # derivative against central differences of the value
    eps, h = 1e-4, 1e-6
    _, d = O.l1_eps_penalty(J, 0.3, eps)
    for (i, j) in [(0, 1), (2, 4), (5, 0), (3, 3)]:
        Jp, Jm = J.copy(), J.copy()
        Jp[i, j] += h
        Jm[i, j] -= h
        fd = (O.l1_eps_penalty(Jp, 0.3, eps)[0][i] - O.l1_eps_penalty(Jm, 0.3, eps)[0][i]) / (2 * h)
        assert abs(fd - d[i, j]) < 1e-8


def test_no_penalty_no_bounds_is_the_mle():
    rec = tiny()
    N, B = rec.n_neurons, rec.n_bins
    Jn, mun, _ = O.newton_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau)
    assert np.abs(Jn).max() < 20  # a well-posed case
    J, mu, res = O.penalized_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, alpha=0.0)
    assert np.abs(J - Jn).max() < 1e-5 and np.abs(mu - mun).max() < 1e-6


@pytest.mark.parametrize("alpha", [0.3, 2.0])
def test_penalised_optimum_satisfies_kkt(alpha):
    rec = tiny()
    N, B = rec.n_neurons, rec.n_bins
    jmax, rmin, rmax = 1.5, 0.001, 8.0
    J, mu, _ = O.penalized_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, alpha=alpha, eps=1e-8,
                               j_max=jmax, rate_min=rmin, rate_max=rmax)
    r = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu)
    _, dpen = O.l1_eps_penalty(J, alpha, 1e-8)
    gJ = r["gJ"] - dpen          # gradient of the penalised objective (maximised)
    gmu = r["gmu"]
    scale = np.abs(O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, np.zeros((N, N)),
                            np.zeros(N))["gJ"]).max()
    tol = 1e-5 * scale
    at_hi_J, at_lo_J = J >= jmax - 1e-9, J <= -jmax + 1e-9
    free = ~(at_hi_J | at_lo_J)
    # entries pinned near zero by the penalty sit where |dL/dJ| <= alpha
    assert np.all(np.abs(gJ[free]) <= tol + 1e-3 * alpha)
    assert np.all(gJ[at_hi_J] >= -tol) and np.all(gJ[at_lo_J] <= tol)
    lo, hi = math.log(rmin), math.log(rmax)
    at_hi_m, at_lo_m = mu >= hi - 1e-9, mu <= lo + 1e-9
    assert at_hi_m.any()  # the rate cap binds for the fast neurons
    assert np.all(gmu[at_hi_m] >= -tol) and np.all(gmu[at_lo_m] <= tol)
    assert np.all(np.abs(gmu[~(at_hi_m | at_lo_m)]) <= tol)


def test_strong_penalty_shrinks_every_coupling():
    rec = tiny()
    N, B = rec.n_neurons, rec.n_bins
    # dL/dJ at the uncoupled optimum bounds the penalty needed to keep J = 0
    q = np.bincount(rec.neurons, minlength=N)
    mu0 = np.log(q / (B * rec.dt))
    g0 = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, np.zeros((N, N)), mu0)["gJ"]
    alpha = 2.0 * np.abs(g0).max()
    J, mu, _ = O.penalized_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, alpha=alpha, eps=1e-10)
    off = ~np.eye(N, dtype=bool)
    assert np.abs(J[off]).max() < 1e-3
    # and the base rates are then the uncoupled MLE up to the self-terms
    assert np.isfinite(mu).all()
