"""Writes tests/golden/events_config2_rows.json: the oracle's continuous-time
L_i, dL/dmu_i and the full gradient row dL/dJ_i. for six rows of config 2 in
continuous time (the balanced N = 1000 network, 3600 s, seed 0, every spike
placed uniformly inside its 1 ms bin by synth.event_times(rec, seed=0):
23.8 M network events), at two parameter points:
  "bf16"  J = the simulated weights rounded to BF16 (round to nearest even),
          mu = the simulated baselines (what the BF16 event grid evaluates);
  "zero"  J = 0, mu = 0.
L is separable over rows (Sec. 2.2), so the rows of continuous_eval are exact
references on their own; they come from the oracle's continuous_eval_rows
(Eq. (7)-(8), (10), (12), (14)).  Calls only the oracle and the input
generator.

Run from the repository root (about ten minutes on 8 cores):
    python tests/golden/make_events_full_rows.py
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

OUT = os.path.join(ROOT, "tests", "golden", "events_config2_rows.json")
ROWS = [0, 257, 500, 799, 800, 999]


def bf16_rne(x):
    """Round float64 values to BF16 (via float32, both round to nearest even)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def main():
    rec = synth.cached("config2", seed=0, B=3_600_000)
    N = rec.n_neurons
    times, neu = synth.event_times(rec, seed=0)
    T0, T1 = 0.0, rec.T
    t0 = time.time()
    points = {"bf16": (bf16_rne(rec.J), rec.mu.copy()), "zero": (np.zeros((N, N)), np.zeros(N))}
    out = {}
    for tag, (J, mu) in points.items():
        r = O.continuous_eval_rows(times, neu, N, T0, T1, rec.tau, J, mu, ROWS)
        out[tag] = dict(ll_rows=[repr(float(v)) for v in r["ll_rows"]],
                        gmu=[repr(float(v)) for v in r["gmu"]],
                        gJ=[[repr(float(v)) for v in row] for row in r["gJ"]])
        print(f"[{time.time() - t0:6.0f} s] {tag}: L_i {r['ll_rows']}", flush=True)
    doc = {
        "_what": "continuous-time L_i, dL/dmu_i, dL/dJ_i. (Eq. (7)-(8), (10), (12), (14)) of sampled rows of "
                 "config 2 in continuous time, by the oracle's continuous_eval_rows",
        "recording": dict(generator="synth.cached('config2', seed=0, B=3600000); synth.event_times(rec, seed=0)",
                          n_neurons=N, n_events=int(times.shape[0]), T0=T0, T1=T1, tau=rec.tau,
                          time_sum=repr(float(np.sum(times))), neuron_sum=int(np.sum(neu.astype(np.int64)))),
        "rows": ROWS,
        "points": out,
        "seconds": time.time() - t0,
        "command": "python tests/golden/make_events_full_rows.py",
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
