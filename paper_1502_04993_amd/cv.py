"""Cross-validation scans over the kernel time constant, the transmission
delay and the penalty (Sec. 2.4, 2.5 and Sec. 3.2, Fig. 4: fit on a training
part of the recording, score the fitted parameters by the likelihood of a
held-out validation part, scan the hyper-parameters over a grid).

The recording is split in time: bins [0, B_t) train, [B_t, B) validate.  For
every grid point the training context is fitted (all grid points that share a
penalty are fitted together, as one batch: one graph replay per ascent step
for all of them), and the validation log-likelihood of row i is

    L_i^val(theta) = L_i(theta; [0, B)) - L_i(theta; [0, B_t)),

exact because the trace is causal: the validation bins see the training
spikes as history, as in the full recording.  Every evaluation and fit runs
in the library's kernels; this module only arranges the contexts.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import Batch, Context


@dataclass
class CVResult:
    taus: List[float]
    alphas: List[float]
    train_bins: int
    # [len(alphas)][len(taus)][N] per-row validation log-likelihoods (with
    # delays: [len(alphas)][len(taus) * len(delays)][N], tau-major)
    val_rows: np.ndarray
    # fitted (J, mu) per grid point, keyed (alpha index, tau index)
    params: Dict[Tuple[int, int], Tuple[np.ndarray, np.ndarray]] = field(default_factory=dict)
    reports: Dict[Tuple[int, int], dict] = field(default_factory=dict)
    # (d, d_self) in bins per delay grid point
    delays: List[Tuple[int, int]] = field(default_factory=lambda: [(0, 0)])

    def point(self, k: int) -> Tuple[float, Tuple[int, int]]:
        """(tau, (d, d_self)) of grid column k."""
        nd = len(self.delays)
        return self.taus[k // nd], self.delays[k % nd]

    @property
    def val(self) -> np.ndarray:
        """Total validation log-likelihood per (alpha, tau)."""
        return self.val_rows.sum(axis=-1)

    def best(self):
        """(alpha, tau) with the largest total validation log-likelihood
        ((alpha, tau, (d, d_self)) when delays were scanned)."""
        a, k = np.unravel_index(np.argmax(self.val), self.val.shape)
        if len(self.delays) == 1:
            return self.alphas[a], self.taus[k]
        tau, dl = self.point(k)
        return self.alphas[a], tau, dl

    def mean_row_peak_tau(self, alpha_index: int = 0) -> float:
        """Mean over rows of the tau at which each row's validation curve peaks
        (the paper averages the peak locations of the per-neuron curves)."""
        peaks = np.argmax(self.val_rows[alpha_index], axis=0)
        return float(np.mean([self.point(k)[0] for k in peaks]))


def _split(bins, neurons, b_train):
    bins = np.asarray(bins, np.int64)
    neurons = np.asarray(neurons, np.int32)
    m = bins < b_train
    return bins[m], neurons[m]


def cv_scan(bins: np.ndarray, neurons: np.ndarray, n_neurons: int, n_bins: int, dt: float,
            taus: Sequence[float], alphas: Sequence[float] = (0.0,), train_frac: float = 0.5,
            precision: str = "fp32", max_iter: int = 500, ftol: float = 0.0, l1_eps: float = 0.0, j_max: float = 0.0,
            rate_min: float = 0.0, rate_max: float = 0.0, device: int = 0,
            delays: Sequence[Tuple[int, int]] = ((0, 0),)) -> CVResult:
    """Fit on the first train_frac of the bins for every (alpha, tau, delay)
    and score each fit on the rest; delays are (d, d_self) pairs in bins.
    Returns a CVResult (per-row validation log-likelihoods, fitted parameters
    and fit reports per grid point)."""
    taus = [float(t) for t in taus]
    alphas = [float(a) for a in alphas]
    dls = [(int(d), int(ds)) for d, ds in delays]
    points = [(tau, dl) for tau in taus for dl in dls]
    b_train = int(round(n_bins * train_frac))
    if not 0 < b_train < n_bins:
        raise ValueError("train_frac must leave bins on both sides of the split")
    tb, tn = _split(bins, neurons, b_train)
    val = np.zeros((len(alphas), len(points), n_neurons))
    out = CVResult(taus, alphas, b_train, val, delays=dls)
    fulls: List[Context] = []
    for tau, (d, ds) in points:
        c = Context(n_neurons, n_bins, dt, precision=precision, device=device)
        if (d, ds) != (0, 0):
            c.set_delays(d, ds)
        c.set_spikes_allow_silent(bins, neurons)
        c.set_kernel(tau)
        fulls.append(c)
    try:
        for ai, alpha in enumerate(alphas):
            trains: List[Context] = []
            try:
                for tau, (d, ds) in points:
                    c = Context(n_neurons, b_train, dt, precision=precision, device=device)
                    if (d, ds) != (0, 0):
                        c.set_delays(d, ds)
                    c.set_spikes(tb, tn)
                    c.set_kernel(tau)
                    trains.append(c)
                batch = Batch(trains)
                try:
                    _, reps = batch.fit(max_iter=max_iter, ftol=ftol, from_zero=True, l1_alpha=alpha, l1_eps=l1_eps,
                                        j_max=j_max, rate_min=rate_min, rate_max=rate_max)
                finally:
                    batch.close()
                for ti, (ct, cf) in enumerate(zip(trains, fulls)):
                    J, mu, _ = ct.get_params()
                    l_train = ct.eval(grad=False)["ll_rows"]
                    cf.set_params(J, mu)
                    l_full = cf.eval(grad=False)["ll_rows"]
                    val[ai, ti] = l_full - l_train
                    out.params[(ai, ti)] = (J, mu)
                    out.reports[(ai, ti)] = reps[ti]
            finally:
                for c in trains:
                    c.close()
    finally:
        for c in fulls:
            c.close()
    return out
