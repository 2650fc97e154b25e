"""Writes tests/golden/config2_optimum_rows.json: the oracle's maximiser of
L_i for 65 rows of the config-2 recording (the balanced N = 1000 network,
3.6e6 bins of 1 ms, seed 0), stratified by type: 51 excitatory rows evenly
spread over 0..799 and 13 inhibitory rows over 800..999, plus row 257.

L is separable over rows (Sec. 2.2) and each row's problem is concave
(App. A), so each row's maximiser is found on its own, here by the oracle's
newton_rows_sub: exact L_i and gradient (Eq. (7), (12)) over all bins at every
iterate, steps scaled by the Hessian of Eq. (18) taken on every 11th time
chunk.  The file keeps each row's (mu_i, J_i), L_i, the iteration count, the
largest gradient component at the result and at the start (from the oracle's
own likelihood, loglik), standard-error estimates from the subsampled Hessian,
and a fingerprint of the recording.  Calls only the oracle and the input
generator.

Run from the repository root (about an hour on 8 cores):
    python tests/golden/make_config2_optimum_rows.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import glm_oracle as O  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "config2_optimum_rows.json")


def stratified_rows():
    exc = np.round(np.linspace(0, 799, 51)).astype(int)
    inh = np.round(np.linspace(800, 999, 13)).astype(int)
    return sorted(set(exc.tolist()) | set(inh.tolist()) | {257})


def fingerprint(rec):
    """Spike count and a checksum of the (bin, neuron) pairs."""
    b = rec.bins.astype(np.int64)
    n = rec.neurons.astype(np.int64)
    return dict(n_spikes=int(b.shape[0]), checksum=int(np.sum((b * 1009 + n) % 1000003)))


def main():
    rows = stratified_rows()
    rec = synth.cached("config2", seed=0, B=3_600_000)
    N, B = rec.n_neurons, rec.n_bins
    t0 = time.time()
    res = O.newton_rows_sub(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, rows, hess_stride=11, refresh=3,
                            log=lambda m: print(f"[{time.time() - t0:7.0f} s] {m}", flush=True))
    secs = time.time() - t0
    J = np.zeros((N, N))
    mu = np.zeros(N)
    for i in rows:
        J[i] = res[i]["J"]
        mu[i] = res[i]["mu"]
    chk = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu, rows=rows)
    q = O.spike_counts(rec.neurons, N)
    start = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, np.zeros((N, N)), np.log(q / (B * rec.dt)),
                     rows=rows)
    rows_out = []
    for k, i in enumerate(rows):
        g = np.concatenate([[chk["gmu"][k]], chk["gJ"][k]])
        g0 = np.concatenate([[start["gmu"][k]], start["gJ"][k]])
        rows_out.append(dict(row=i, mu=repr(res[i]["mu"]), J=[repr(float(v)) for v in res[i]["J"]],
                             ll=repr(res[i]["ll"]), ll_oracle_check=repr(float(chk["ll_rows"][k])),
                             se_mu=float(f"{res[i]['se'][0]:.3g}"),
                             se_J=[float(f"{v:.3g}") for v in res[i]["se"][1:]],
                             iters=res[i]["iters"], max_abs_grad=float(np.abs(g).max()),
                             max_abs_grad_at_start=float(np.abs(g0).max())))
        print(f"row {i}: iters {res[i]['iters']} max|grad| {np.abs(g).max():.3e} "
              f"(start {np.abs(g0).max():.3e})", flush=True)
    doc = {
        "_what": "maximiser (mu_i, J_i) of the grid likelihood (Eq. (7), gradient Eq. (12)) for 65 stratified "
                 "rows of config 2, by the oracle's newton_rows_sub (exact gradient, Hessian of Eq. (18) on "
                 "every 11th chunk); se_* are estimates from that subsampled Hessian",
        "recording": dict(generator="synth.cached('config2', seed=0, B=3600000)", n_neurons=N, n_bins=B,
                          dt=rec.dt, tau=rec.tau, **fingerprint(rec)),
        "rows": rows_out,
        "seconds": secs,
        "command": "python tests/golden/make_config2_optimum_rows.py",
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {OUT} in {secs:.0f} s", flush=True)


if __name__ == "__main__":
    main()
