"""Synthetic workload generator: Philox known answers, determinism, structure."""
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _u32(v):
    return int(v, 16) if isinstance(v, str) else int(v)


def test_philox_known_answers():
    kat = json.load(open(GOLDEN))["philox4x32_10_kat"]["vectors"]
    for v in kat:
        out = synth.philox4x32_10([_u32(c) for c in v["ctr"]], [_u32(k) for k in v["key"]])
        assert [int(x) for x in out] == [_u32(o) for o in v["out"]]


def test_seeded_and_thread_independent():
    N, B = 64, 3000
    J = synth.net_bernoulli(N, 51, 0.2, 0.5, -1.5, 4)
    mu = np.full(N, np.log(8.0))
    b1, n1 = synth.simulate(N, B, 0.001, 0.01, mu, J, 4, threads=1)
    b2, n2 = synth.simulate(N, B, 0.001, 0.01, mu, J, 4, threads=4)
    assert np.array_equal(b1, b2) and np.array_equal(n1, n2)
    b3, n3 = synth.simulate(N, B, 0.001, 0.01, mu, J, 5, threads=4)
    assert not (b3.shape == b1.shape and np.array_equal(b3, b1))
    # sorted by (bin, neuron)
    key = b1 * N + n1
    assert np.all(np.diff(key) > 0)


def test_config1_structure():
    r = synth.config1(0)
    assert r.n_neurons == 50 and r.n_bins == 20_000 and r.n_exc == 40
    off = ~np.eye(50, dtype=bool)
    assert np.all(np.diag(r.J) == 0)
    assert set(np.unique(r.J[:, :40][off[:, :40]])) <= {0.0, 0.5}
    assert set(np.unique(r.J[:, 40:][off[:, 40:]])) <= {0.0, -1.5}
    p_hat = (r.J[off] != 0).mean()
    assert abs(p_hat - 0.2) < 0.03
    rate = r.n_spikes / (50 * r.T)
    assert 3.0 < rate < 10.0
    assert r.counts().min() > 0


def test_fixed_indegree_exact():
    J = synth.net_fixed_indegree(200, 160, 16, 4, 0.2, -1.0, 3)
    assert np.all((J[:, :160] > 0).sum(axis=1) == 16)
    assert np.all((J[:, 160:] < 0).sum(axis=1) == 4)
    assert np.all(np.diag(J) == 0)


def test_balanced_rates_in_range():
    r = synth.balanced(N=300, B=30_000, seed=1)
    rate = r.n_spikes / (300 * r.T)
    assert 5.0 <= rate <= 10.0, rate
    assert np.all(np.diag(r.J) == -5.0)


def test_synfire_structure():
    r = synth.synfire(N=700, B=20_000, seed=2)
    g = r.group_of
    assert (g >= 0).sum() == 500 and np.all(g[g >= 0] < 10)
    assert np.all(g[r.n_exc:] == -1)  # groups are excitatory
    # chain weights only between consecutive groups
    pre = np.where(g == 3)[0]
    post = np.where(g == 4)[0]
    blk = r.J[np.ix_(post, pre)]
    frac = (blk == 0.4).mean()
    assert 0.4 < frac < 0.6
    rate = r.n_spikes / (700 * r.T)
    assert rate < 40.0


def test_config5_sizes():
    sizes = synth.config5_sizes()
    assert len(sizes) == 64
    for r, (kind, N, B, seed) in enumerate(sizes):
        assert seed == 1000 + r
        assert 60_000 <= B <= 600_000
        assert (100 if kind == "balanced" else 625) <= N <= 2000
    assert sum(k == "synfire" for k, *_ in sizes) == 32
