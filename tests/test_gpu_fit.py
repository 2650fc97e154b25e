"""The per-row L-BFGS ascent on the GPU against the oracle's optimum."""
import numpy as np
import pytest

import synth
from oracle import glm_oracle as O

pytestmark = pytest.mark.gpu


def _G():
    import paper_1502_04993_amd as G
    return G


def test_fit_config1_fp64_matches_newton_optimum():
    rec = synth.config1(0)
    N, B = rec.n_neurons, rec.n_bins
    G = _G()
    ctx = G.Context(N, B, rec.dt, precision="fp64")
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    rep = ctx.fit(max_iter=1000, from_zero=True)
    J, mu, tau = ctx.get_params()
    ctx.close()
    print(f"[fit config1 fp64] {rep}", flush=True)
    Jn, mun, _ = O.newton_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau)
    # KKT at the GPU optimum, measured by the oracle (Sec. 2.3.3: expected count = observed)
    r0 = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, np.zeros((N, N)), np.zeros(N))
    r = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu)
    g0 = np.linalg.norm(np.concatenate([r0["gmu"], r0["gJ"].ravel()]))
    g = np.linalg.norm(np.concatenate([r["gmu"], r["gJ"].ravel()]))
    print(f"  |grad(theta_gpu)|/|grad(0)| = {g / g0:.3e}  max|J-Jn| = {np.abs(J - Jn).max():.3e} "
          f"max|mu-mun| = {np.abs(mu - mun).max():.3e}", flush=True)
    assert rep["converged"]
    assert g <= 1e-6 * g0
    assert np.abs(J - Jn).max() < 1e-5 and np.abs(mu - mun).max() < 1e-5
    lab_g = O.classify(J)
    lab_o = O.classify(Jn)
    assert np.array_equal(lab_g, lab_o)


def test_fit_mu_warm_start_and_zero_iterations():
    rec = synth.config1(1)
    N, B = rec.n_neurons, rec.n_bins
    G = _G()
    ctx = G.Context(N, B, rec.dt, precision="fp64")
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    rep = ctx.fit(max_iter=0, from_zero=True, warm_start_mu=True)
    J, mu, _ = ctx.get_params()
    q = np.bincount(rec.neurons, minlength=N)
    assert rep["status"] == 1 and rep["iters"] == 0  # NOT_CONVERGED, nothing done
    assert np.allclose(np.exp(mu), q / (B * rec.dt), rtol=1e-14) and np.all(J == 0)
    ctx.close()


def _standard_errors(rec, J, mu):
    """sqrt(diag(-H^-1)) per row at (J, mu), H the row Hessian of Eq. (18)."""
    N, B = rec.n_neurons, rec.n_bins
    X = O.dense_trace(rec.bins, rec.neurons, N, B, rec.dt, rec.tau)
    A = np.hstack([np.ones((B, 1)), X])
    se = np.zeros((N, N))
    for i in range(N):
        lam = np.exp(mu[i] + X @ J[i])
        H = rec.dt * (A.T * lam) @ A
        se[i] = np.sqrt(np.diag(np.linalg.inv(H))[1:])
    return se


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_fit_reduced_precision_reaches_oracle_optimum(prec):
    rec = synth.config1(0)
    N, B = rec.n_neurons, rec.n_bins
    G = _G()
    ctx = G.Context(N, B, rec.dt, precision=prec)
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    rep = ctx.fit(max_iter=1000, from_zero=True)
    J, mu, _ = ctx.get_params()
    ctx.close()
    Jn, mun, _ = O.newton_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau)
    err = np.abs(J - Jn).max()
    se = _standard_errors(rec, Jn, mun)
    zmax = float(np.max(np.abs(J - Jn) / se))
    print(f"[fit config1 {prec}] {rep} max|J-Jn|={err:.3e} max|J-Jn|/SE={zmax:.3f}", flush=True)
    # BF16 evaluates the likelihood at bf16(J) with a stochastically rounded
    # trace, so its maximum sits a little away from the exact one; the bound is
    # a fraction of the MLE's own standard error (Hessian of Eq. (18)), the
    # resolution the data allow (0.25 .. 2 at this size)
    if prec == "fp32":
        assert err < 1e-3
    else:
        assert zmax < 0.5
    if prec == "fp32":
        assert np.array_equal(O.classify(J), O.classify(Jn))
    else:
        # labels may differ only for entries this close to a k-means boundary
        lab_g, lab_o = O.classify(J), O.classify(Jn)
        _, c = O.kmeans3(Jn[~np.eye(N, dtype=bool)])
        bounds = np.array([(c[0] + c[1]) / 2, (c[1] + c[2]) / 2])
        near = np.min(np.abs(Jn[..., None] - bounds[None, None, :]), axis=-1) < 2 * err
        assert np.all((lab_g == lab_o) | near)


def test_bf16_fit_with_fp32_polish_matches_oracle_classification():
    rec = synth.config1(0)
    N, B = rec.n_neurons, rec.n_bins
    G = _G()
    ctx = G.Context(N, B, rec.dt, precision="bf16")
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    rep = ctx.fit(max_iter=1000, from_zero=True, polish="fp32")
    J, mu, _ = ctx.get_params()
    assert ctx.precision == "bf16"
    ctx.close()
    Jn, mun, _ = O.newton_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau)
    err = np.abs(J - Jn).max()
    print(f"[fit config1 bf16+fp32 polish] {rep} max|J-Jn|={err:.3e}", flush=True)
    assert err < 1e-3
    assert np.array_equal(O.classify(J), O.classify(Jn))


def test_continuation_with_kept_history_and_refusals():
    """A BF16 ascent continued in FP64 from its L-BFGS pairs (keep_history)
    reaches the oracle's Newton optimum like a continuation from an empty
    history; keeping needs pairs of the same recording, kernel and lbfgs_m."""
    rec = synth.config1(0)
    N, B = rec.n_neurons, rec.n_bins
    G = _G()
    Jn, mun, _ = O.newton_fit(rec.bins, rec.neurons, N, B, rec.dt, rec.tau)
    out = {}
    for keep in (False, True):
        ctx = G.Context(N, B, rec.dt, precision="bf16")
        ctx.set_spikes(rec.bins, rec.neurons)
        ctx.set_kernel(rec.tau)
        if keep:
            with pytest.raises(G.GlmrError) as e:  # no ascent yet
                ctx.fit(max_iter=5, keep_history=True)
            assert e.value.status == G.L.GLMR_ESTATE
        ctx.fit(max_iter=1000, from_zero=True)
        ctx.set_precision("fp64")
        if keep:
            with pytest.raises(G.GlmrError) as e:  # pairs of another history length
                ctx.fit(max_iter=5, keep_history=True, lbfgs_m=10)
            assert e.value.status == G.L.GLMR_ESTATE
        rep = ctx.fit(max_iter=1000, keep_history=keep)
        J, mu, _ = ctx.get_params()
        out[keep] = rep
        err = max(np.abs(J - Jn).max(), np.abs(mu - mun).max())
        print(f"[fit config1 bf16 -> fp64, keep_history={keep}] {rep} max err {err:.3e}", flush=True)
        assert rep["converged"] and err < 1e-5
        assert np.array_equal(O.classify(J), O.classify(Jn))
        if keep:
            ctx.set_kernel(1.2 * rec.tau)  # another objective: the pairs are dropped
            with pytest.raises(G.GlmrError) as e:
                ctx.fit(max_iter=5, keep_history=True)
            assert e.value.status == G.L.GLMR_ESTATE
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_graph_replays_match_eager_steps(prec):
    """The captured ascent step replayed k times gives bitwise the parameters
    that k eagerly launched steps give, for several k (each fit re-captures;
    the host reads the active-row counter between replays)."""
    import os
    rec = synth.config1(0)
    N, B = rec.n_neurons, rec.n_bins
    G = _G()
    old = os.environ.get("GLMR_NO_GRAPH")
    try:
        for k in (1, 2, 3, 5, 8, 25):
            out = []
            for flag in ("1", "0"):
                os.environ["GLMR_NO_GRAPH"] = flag
                ctx = G.Context(N, B, rec.dt, precision=prec)
                ctx.set_spikes(rec.bins, rec.neurons)
                ctx.set_kernel(rec.tau)
                rep = ctx.fit(max_iter=k, from_zero=True)
                J, mu, _ = ctx.get_params()
                ctx.close()
                out.append((J, mu, rep["iters"], rep["ll"]))
            assert out[0][2] == out[1][2] == k
            assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
            assert out[0][3] == out[1][3]
    finally:
        if old is None:
            os.environ.pop("GLMR_NO_GRAPH", None)
        else:
            os.environ["GLMR_NO_GRAPH"] = old
