"""The event grid's interval integrals (Eq. (10), (14)) as the library
computes them, on the CPU: the same host/device code the kernels run,
reached through glmr_ei_interval, against the exponential integral and the
exponential evaluated to 40 digits by mpmath.  Covers every branch of the
evaluation (the midpoint Taylor expansion of short intervals, the |D| <= 2
series, the near-cancelling Gauss-Legendre branch,
the direct difference of Ei for either sign and for large arguments) and the
limits delta -> 0, delta -> large, D -> 0."""
import numpy as np
import pytest

mp = pytest.importorskip("mpmath")


def _ref(D, delta):
    mp.mp.dps = 40
    Dm, dm = mp.mpf(D), mp.mpf(delta)
    xi = mp.e ** (-dm)
    if D == 0:
        return dm, 1 - xi
    return mp.ei(Dm) - mp.ei(Dm * xi), (mp.e ** Dm - mp.e ** (Dm * xi)) / Dm


def _cases():
    rng = np.random.default_rng(7)
    D = np.concatenate([rng.uniform(-3, 3, 300), rng.uniform(-40, 60, 300),
                        [0.0, 1e-12, -1e-12, 2.0, -2.0, 2.0 + 1e-9, -2.0 - 1e-9, 40.0, 41.0, -1.0, 200.0]])
    delta = 10 ** rng.uniform(-9, 2.6, D.shape[0])
    delta[:40] = 10 ** rng.uniform(-12, -6, 40)
    # the short intervals between the events of a large network (the
    # midpoint-Taylor branch and its boundary delta max(1, |u|) = 0.1)
    Ds = rng.uniform(-12, 12, 400)
    ds = 10 ** rng.uniform(-6, -0.9, 400)
    return list(zip(D.tolist(), delta.tolist())) + list(zip(Ds.tolist(), ds.tolist()))


def test_interval_integrals_match_mpmath_in_every_branch():
    import paper_1502_04993_amd as G
    worst_f = worst_h = 0.0
    for D, delta in _cases():
        F, H = G.glmr_ei_interval(D, delta)
        Fr, Hr = _ref(D, delta)
        worst_f = max(worst_f, float(abs((F - Fr) / Fr)))
        worst_h = max(worst_h, float(abs((H - Hr) / Hr)))
    assert worst_f < 5e-14 and worst_h < 5e-14, (worst_f, worst_h)


def test_interval_integrals_limits():
    import paper_1502_04993_amd as G
    # zero length: nothing
    assert G.glmr_ei_interval(1.3, 0.0) == (0.0, 0.0)
    # D = 0: F = delta, H = 1 - e^{-delta}
    F, H = G.glmr_ei_interval(0.0, 0.37)
    assert F == pytest.approx(0.37, rel=1e-15) and H == pytest.approx(-np.expm1(-0.37), rel=1e-15)
    # short interval: F -> e^D delta, H -> e^D delta
    F, H = G.glmr_ei_interval(0.8, 1e-10)
    assert F == pytest.approx(np.exp(0.8) * 1e-10, rel=1e-9) and H == pytest.approx(np.exp(0.8) * 1e-10, rel=1e-9)
    # additivity over a split interval (the spike-free slots rely on it)
    for D in (-5.0, -0.4, 0.9, 3.5):
        a, b = 0.3, 0.45
        F1, H1 = G.glmr_ei_interval(D, a)
        F2, H2 = G.glmr_ei_interval(D * np.exp(-a), b)
        F, H = G.glmr_ei_interval(D, a + b)
        assert F1 + F2 == pytest.approx(F, rel=1e-13)
        assert H1 + np.exp(-a) * H2 == pytest.approx(H, rel=1e-13)


def _tier_f32(D, delta):
    """Which tier of the FP32 chain takes (D, delta): 0 the midpoint expansion,
    1 the 6-point quadrature, 2 the FP64 evaluation."""
    D = float(np.float32(D))
    u = D * float(np.float32(np.exp(-0.5 * delta)))
    if float(np.float32(delta)) * max(1.0, abs(u)) <= 0.35:
        return 0
    return 1 if (delta <= 0.5 and abs(D) * delta <= 1.0) else 2


def test_fp32_interval_chain_matches_mpmath_in_every_tier():
    # the BF16 event grid's integrals: an FP32 potential, FP32 arithmetic;
    # relative error within a few units of 2^-24 per unit of |u| (the
    # exponential of a rounded argument), in each of the three tiers
    import paper_1502_04993_amd as G
    rng = np.random.default_rng(11)
    D = np.concatenate([rng.uniform(-3, 3, 400), rng.uniform(-12, 12, 400), rng.uniform(-30, 30, 200),
                        [0.0, 1.0, -1.0, 1e-7]])
    delta = np.concatenate([10 ** rng.uniform(-6, -0.3, 800), 10 ** rng.uniform(-3, 1.5, 200),
                            [0.25, 0.25, 0.25, 0.3]])
    seen = [0, 0, 0]
    worst = 0.0
    for d_, dl in zip(D.tolist(), delta.tolist()):
        Df = float(np.float32(d_))
        F, H = G.glmr_ei_interval_f32(Df, dl)
        Fr, Hr = _ref(Df, dl)
        scale = 1e-7 * (8.0 + abs(Df))
        ef, eh = float(abs((F - Fr) / Fr)), float(abs((H - Hr) / Hr))
        seen[_tier_f32(Df, dl)] += 1
        worst = max(worst, ef / scale, eh / scale)
        assert ef <= scale and eh <= scale, (Df, dl, ef, eh)
    assert min(seen) >= 20, seen
    print(f"[fp32 chain] tiers {seen} worst {worst:.3f} of the bound")


def test_fp32_expansion_at_its_bound_and_degenerate_intervals():
    import paper_1502_04993_amd as G
    # on the bound delta max(1, |u|) = 0.35 from both sides: the expansion's
    # truncation stays far below FP32 rounding
    for D in (-6.0, -1.0, 0.5, 1.0, 4.0):
        for dl in np.linspace(0.25, 0.45, 41):
            u = D * np.exp(-dl / 2)
            F, H = G.glmr_ei_interval_f32(D, dl)
            Fr, Hr = _ref(D, dl)
            assert abs((F - Fr) / Fr) < 1e-6 and abs((H - Hr) / Hr) < 1e-6, (D, dl, u)
    assert G.glmr_ei_interval_f32(2.5, 0.0) == (0.0, 0.0)
    F, H = G.glmr_ei_interval_f32(0.0, 0.1)
    assert F == pytest.approx(0.1, rel=2e-7) and H == pytest.approx(-np.expm1(-0.1), rel=2e-7)
