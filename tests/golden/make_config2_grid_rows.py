"""Writes tests/golden/config2_grid_rows.json: the oracle's grid L_i, dL/dmu_i
and gradient row dL/dJ_i. (Eq. (7), (12)) for five rows of the config-2
recording (the balanced N = 1000 network, 3.6e6 bins of 1 ms, seed 0) at the
parameters that the bench's BF16/FP32 and FP8 lines evaluate:
  "bf16"  J = the simulated weights rounded to BF16 (round to nearest even;
          exact in FP32 as well), mu = the simulated baselines;
  "fp8"   J rounded as the FP8 path represents it: per row a power-of-two
          scale 2^floor(log2(448 / max_j |J_ij|)), the scaled FP32 value
          rounded to the nearest e4m3 value (ties to even).
L is separable over rows (Sec. 2.2), so a few rows are exact references at
full size.  Each point keeps its rounded weight rows (J_rows) with the
results.  The bench reports its gradient error against these rows (it sets
the stored weight rows, evaluates, and compares); it reads this file and does
not run the oracle.  Calls only the oracle and the
input generator.

Run from the repository root (a few minutes on 8 cores):
    python tests/golden/make_config2_grid_rows.py
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

OUT = os.path.join(ROOT, "tests", "golden", "config2_grid_rows.json")
ROWS = [0, 257, 799, 800, 999]


def bf16_rne(x):
    """Round float64 values to BF16 (via float32, both round to nearest even)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def e4m3_rne(y):
    """Nearest OCP e4m3 value (ties to even) of |y| <= 448: 3 mantissa bits,
    exponents down to 2^-6, subnormal step 2^-9."""
    y = np.asarray(y, np.float64)
    a = np.abs(y)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -6)))
    step = 2.0 ** (e - 3)
    return np.sign(y) * np.round(a / step) * step


def fp8_rows(J):
    out = np.zeros_like(J)
    for i in range(J.shape[0]):
        m = np.float32(np.max(np.abs(J[i])))
        sc = 1.0
        if m > 0:
            _, e = np.frexp(np.float32(448.0) / m)
            sc = 2.0 ** (int(e) - 1)
        y = (J[i].astype(np.float32) * np.float32(sc)).astype(np.float64)
        out[i] = e4m3_rne(y) / sc
    return out


def main():
    rec = synth.cached("config2", seed=0, B=3_600_000)
    N, B = rec.n_neurons, rec.n_bins
    t0 = time.time()
    out = {}
    for tag, J in (("bf16", bf16_rne(rec.J)), ("fp8", fp8_rows(rec.J))):
        r = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, rec.mu, rows=ROWS)
        out[tag] = dict(J_rows=[[repr(float(v)) for v in J[i]] for i in ROWS],
                        ll_rows=[repr(float(v)) for v in r["ll_rows"]],
                        gmu=[repr(float(v)) for v in r["gmu"]],
                        gJ=[[repr(float(v)) for v in row] for row in r["gJ"]])
        print(f"[{time.time() - t0:6.0f} s] {tag}: L_i {r['ll_rows']}", flush=True)
    b = rec.bins.astype(np.int64)
    n = rec.neurons.astype(np.int64)
    doc = {
        "_what": "grid L_i, dL/dmu_i, dL/dJ_i. (Eq. (7), (12)) of sampled rows of config 2 at the BF16- and "
                 "FP8-rounded simulated weights, by the oracle's loglik",
        "recording": dict(generator="synth.cached('config2', seed=0, B=3600000)", n_neurons=N, n_bins=B,
                          dt=rec.dt, tau=rec.tau, n_spikes=int(b.shape[0]),
                          checksum=int(np.sum((b * 1009 + n) % 1000003))),
        "rows": ROWS,
        "points": out,
        "seconds": time.time() - t0,
        "command": "python tests/golden/make_config2_grid_rows.py",
    }
    with open(OUT, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
