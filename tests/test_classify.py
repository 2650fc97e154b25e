"""The product's classification (Sec. 3.3) against the oracle's k-means and
its error rate, on synthetic weight matrices (host logic, CPU)."""
import numpy as np
import pytest

import synth
from oracle import glm_oracle as O


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_classify_matches_oracle(seed):
    from paper_1502_04993_amd.classify import classify, misclassification
    rng = np.random.default_rng(seed)
    rec = synth.balanced(N=120, B=1000, seed=seed) if seed < 2 else None
    if rec is not None:
        Jt = rec.J
    else:
        Jt = np.where(rng.random((80, 80)) < 0.2, rng.choice([0.5, -1.5], (80, 80)), 0.0)
    J = Jt + rng.normal(0, 0.15, Jt.shape)  # a noisy reconstruction
    a, b = classify(J), O.classify(J)
    assert np.array_equal(a, b)
    m = misclassification(a, Jt)
    r = O.mer(b, Jt)
    assert m["errors"] == r["errors"] and m["mer"] == r["mer"] and m["mer_n2"] == r["mer_n2"]


def test_classify_exact_weights_have_no_errors():
    from paper_1502_04993_amd.classify import classify, misclassification
    Jt = np.zeros((30, 30))
    Jt[::3, 1::4] = 0.5
    Jt[1::5, ::2] = -1.0
    np.fill_diagonal(Jt, -5.0)
    assert misclassification(classify(Jt), Jt)["errors"] == 0
