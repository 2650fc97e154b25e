"""Element-wise comparison of a GPU evaluation with the FP64 oracle.

Four errors are measured and each is asserted against its own bound:
  ll    |L - L_or| / |L_or|                       (total, Eq. (7))
  row   max_i |L_i - L_i,or| / s_i                (per row; L is separable, Sec. 2.2),
                                                  s_i = max(|L_i,or|, 0.1 I_i) with I_i the
                                                  oracle's integral term of row i: a row whose
                                                  two terms nearly cancel (L_i ~ 0, as for a
                                                  rate near e per second) is measured against
                                                  the size of its terms
  grad  ||g - g_or||_2 / ||g_or||_2               over (dL/dmu, dL/dJ)   (Eq. (12))
  gmax  max |g - g_or| / ||g_or||_inf             (a single wrong entry or a wrong strip
                                                   of a tile shows here, not in the 2-norm)
"""
import sys

import numpy as np


def errors(got, ref, rows=None):
    """Errors of `got` (a Context.eval dict, all rows) against `ref` (an oracle
    dict, restricted to `rows` when given)."""
    sel = slice(None) if rows is None else np.asarray(rows)
    lr = np.asarray(got["ll_rows"])[sel]
    out = {}
    if rows is None:
        out["ll"] = abs(got["ll"] - ref["ll"]) / abs(ref["ll"])
    scale = np.abs(np.asarray(ref["ll_rows"]))
    if ref.get("integral_term") is not None:
        scale = np.maximum(scale, 0.1 * np.abs(np.asarray(ref["integral_term"])))
    out["row"] = float(np.max(np.abs(lr - ref["ll_rows"]) / np.maximum(scale, 1e-300)))
    if got.get("gJ") is not None and ref.get("gJ") is not None:
        g = np.concatenate([np.asarray(got["gmu"])[sel], np.asarray(got["gJ"])[sel].ravel()])
        gr = np.concatenate([np.asarray(ref["gmu"]), np.asarray(ref["gJ"]).ravel()])
        out["grad"] = float(np.linalg.norm(g - gr) / max(np.linalg.norm(gr), 1e-300))
        out["gmax"] = float(np.max(np.abs(g - gr)) / max(np.max(np.abs(gr)), 1e-300))
    return out


def check(tag, got, ref, tol, rows=None):
    """Print the errors, then assert each against tol (a dict with the keys
    of errors(); a missing key is not checked)."""
    e = errors(got, ref, rows)
    print(f"[{tag}] " + " ".join(f"{k}={v:.3e}" for k, v in e.items()), flush=True)
    sys.stdout.flush()
    bad = {k: (v, tol[k]) for k, v in e.items() if k in tol and not v <= tol[k]}
    assert not bad, f"{tag}: errors above their bounds (error, bound): {bad}"
    return e
