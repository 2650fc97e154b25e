"""Penalised, bound-constrained fits on the GPU (Eq. (16)-(17), bounds of
Sec. 2.6.3) against the oracle's L-BFGS-B optimum (needs an MI355X).

The penalised objective is strictly concave and the box convex, so the
maximiser is unique: the GPU fit must reach the oracle's objective value,
its parameters, and the KKT conditions of the bounded problem.
"""
import math

import numpy as np
import pytest

import synth
from oracle import glm_oracle as O

pytestmark = pytest.mark.gpu

ALPHA, EPS, JMAX, RMIN, RMAX = 0.3, 1e-8, 1.5, 0.001, 8.0


def _case():
    return synth.balanced(N=10, B=30000, in_frac=0.3, seed=3)


def _objective(rec, J, mu, alpha):
    r = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, rec.tau, J, mu)
    pen, dpen = O.l1_eps_penalty(J, alpha, EPS)
    return r["ll_rows"] - pen, r["gJ"] - dpen, r["gmu"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_penalised_bounded_fit_reaches_oracle_optimum(prec):
    import paper_1502_04993_amd as G
    rec = _case()
    N, B = rec.n_neurons, rec.n_bins
    Jo, muo, _ = O.penalized_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, alpha=ALPHA, eps=EPS,
                                 j_max=JMAX, rate_min=RMIN, rate_max=RMAX)
    ctx = G.Context(N, B, rec.dt, precision=prec)
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    rep = ctx.fit(max_iter=3000, from_zero=True, l1_alpha=ALPHA, l1_eps=EPS, j_max=JMAX, rate_min=RMIN,
                  rate_max=RMAX)
    J, mu, _ = ctx.get_params()
    ctx.close()
    fo, _, _ = _objective(rec, Jo, muo, ALPHA)
    fg, gJ, gmu = _objective(rec, J, mu, ALPHA)
    print(f"[penalised fit {prec}] {rep} objective gpu {fg.sum():.10f} oracle {fo.sum():.10f} "
          f"max|J-Jo|={np.abs(J - Jo).max():.2e} max|mu-muo|={np.abs(mu - muo).max():.2e}", flush=True)
    # inside the box
    assert np.all(np.abs(J) <= JMAX + 1e-12)
    assert np.all(mu >= math.log(RMIN) - 1e-12) and np.all(mu <= math.log(RMAX) + 1e-12)
    # the same maximum, row by row
    assert np.all(fg >= fo - 1e-7 * np.abs(fo))
    assert np.abs(J - Jo).max() < 2e-3 and np.abs(mu - muo).max() < 1e-4
    # KKT of the bounded problem (gradient of the maximised objective)
    at_hi, at_lo = J >= JMAX - 1e-12, J <= -JMAX + 1e-12
    assert np.all(gJ[at_hi] >= -1e-3) and np.all(gJ[at_lo] <= 1e-3)
    mu_hi = mu >= math.log(RMAX) - 1e-12
    assert mu_hi.any() and np.all(gmu[mu_hi] >= -1e-3)


def test_rate_bound_alone_holds_capped_rows_at_the_bound():
    import paper_1502_04993_amd as G
    rec = _case()
    N, B = rec.n_neurons, rec.n_bins
    ctx = G.Context(N, B, rec.dt, precision="fp64")
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    ctx.fit(max_iter=2000, from_zero=True, rate_max=RMAX)
    J, mu, _ = ctx.get_params()
    ctx.close()
    Jo, muo, _ = O.penalized_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, alpha=0.0, rate_max=RMAX)
    capped = muo >= math.log(RMAX) - 1e-9
    assert capped.any()
    assert np.all(np.abs(mu[capped] - math.log(RMAX)) < 1e-12)
    assert np.abs(J - Jo).max() < 1e-4 and np.abs(mu - muo).max() < 1e-6
