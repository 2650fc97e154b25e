"""E/I/none classification of reconstructed couplings and its error rate
(Sec. 3.3, Eq. (20)).

The off-diagonal weights are clustered in one dimension into three groups by
Lloyd's k-means started from (min, 0, max) and iterated to a fixed point; the
lowest centroid is "inhibitory", the middle one "unconnected", the highest
"excitatory".  Self-couplings (refractoriness, Sec. 3.1) are left out.  The
misclassification error rate counts the off-diagonal pairs whose class
differs from the sign of the generating weight, over N(N - 1) pairs and over
N^2 (the denominator of the paper's tables).  Host arithmetic on the N^2
fitted weights; nothing here is on the likelihood's path.
"""
from __future__ import annotations

import numpy as np

INHIBITORY, UNCONNECTED, EXCITATORY = 0, 1, 2


def kmeans3(values, max_iter: int = 1000):
    """Labels (0 low, 1 middle, 2 high) and centroids of 1-D k-means, k = 3.
    Sorting the values makes each assignment step two boundary searches."""
    v = np.sort(np.asarray(values, dtype=np.float64).ravel())
    if v.size == 0:
        return np.zeros(0, np.int64), np.zeros(3)
    c = np.array([v[0], 0.0, v[-1]])
    csum = np.concatenate([[0.0], np.cumsum(v)])
    cuts = None
    for _ in range(max_iter):
        # points nearer the lower of two neighbouring centroids go below the
        # midpoint (ties to the lower cluster, as argmin over distances does)
        order = np.argsort(c, kind="stable")
        cs = c[order]
        b1 = np.searchsorted(v, 0.5 * (cs[0] + cs[1]), side="right")
        b2 = np.searchsorted(v, 0.5 * (cs[1] + cs[2]), side="right")
        new = (b1, b2)
        if new == cuts:
            break
        cuts = new
        for k, (lo, hi) in enumerate(((0, b1), (b1, b2), (b2, v.size))):
            if hi > lo:
                cs[k] = (csum[hi] - csum[lo]) / (hi - lo)
        c = cs
    c = np.sort(c)
    x = np.asarray(values, dtype=np.float64).ravel()
    b1 = 0.5 * (c[0] + c[1])
    b2 = 0.5 * (c[1] + c[2])
    labels = np.where(x <= b1, INHIBITORY, np.where(x <= b2, UNCONNECTED, EXCITATORY))
    return labels.astype(np.int64), c


def classify(J: np.ndarray) -> np.ndarray:
    """Class of every off-diagonal entry of J (diagonal = -1)."""
    J = np.asarray(J, dtype=np.float64)
    N = J.shape[0]
    off = ~np.eye(N, dtype=bool)
    lab, _ = kmeans3(J[off])
    out = np.full((N, N), -1, dtype=np.int64)
    out[off] = lab
    return out


def misclassification(labels: np.ndarray, J_true: np.ndarray) -> dict:
    """Errors against the signs of the generating weights (Eq. (20))."""
    J_true = np.asarray(J_true, dtype=np.float64)
    N = J_true.shape[0]
    off = ~np.eye(N, dtype=bool)
    truth = np.where(J_true > 0, EXCITATORY, np.where(J_true < 0, INHIBITORY, UNCONNECTED))
    wrong = off & (labels != truth)
    n = int(wrong.sum())
    return dict(errors=n, mer=n / (N * (N - 1)), mer_n2=n / (N * N))
