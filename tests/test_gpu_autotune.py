"""Tile shapes of the resident BF16 contractions and the autotuner (needs an MI355X).

Kernel U accumulates every V in the same k order whatever the tile shape;
the shapes differ only in how the FP32 sums of exp(V) over a wave's bins
are grouped before the FP64 sums, and kernel G's in how its FP32 partials
are grouped over time.  So all shapes agree far inside the BF16 tolerance.
Shapes 0-6 are the row-major kernels (GLMR_XFRAG=0), 7-10 the fragment-major
ones (the default for BF16 on the uniform grid).
"""
import os

import numpy as np
import pytest

import synth
from parity_check import check
from test_gpu_parity import TOL
from oracle import glm_oracle as O

pytestmark = pytest.mark.gpu

N_SHAPES = 11
FRAG = (7, 8, 9, 10)


def _ctx(rec, shape=None, frag=True):
    import paper_1502_04993_amd as G
    saved = {k: os.environ.pop(k, None) for k in ("GLMR_RES_SHAPE", "GLMR_XFRAG")}
    if shape is not None:
        os.environ["GLMR_RES_SHAPE"] = f"{shape},{shape}"
        frag = shape in FRAG
    if not frag:
        os.environ["GLMR_XFRAG"] = "0"
    try:
        ctx = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision="bf16")
    finally:
        for k, v in saved.items():
            os.environ.pop(k, None)
            if v is not None:
                os.environ[k] = v
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    return ctx


def test_every_shape_agrees_and_matches_oracle():
    rec = synth.balanced(N=512, B=40_000, seed=21)
    J, mu = rec.J, rec.mu
    import torch
    Jb = torch.tensor(J).to(torch.bfloat16).to(torch.float64).numpy()
    ref = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, rec.tau, Jb, mu)
    gref = np.concatenate([ref["gmu"], ref["gJ"].ravel()])
    lls, grads = [], []
    for k in range(N_SHAPES):
        ctx = _ctx(rec, k)
        ctx.set_params(Jb, mu)
        r = ctx.eval(grad=True)
        assert ctx.query()["trace_resident"] and ctx.query()["trace_frag"] == (k in FRAG)
        ctx.close()
        g = np.concatenate([r["gmu"], r["gJ"].ravel()])
        check(f"shape {k}", r, ref, TOL["bf16"])
        lls.append(r["ll"])
        grads.append(g)
    assert all(abs(l - lls[0]) <= 1e-9 * abs(lls[0]) for l in lls)
    for g in grads[1:]:
        assert np.linalg.norm(g - grads[0]) / np.linalg.norm(grads[0]) < 1e-5


@pytest.mark.parametrize("shape", [0, 3, 4, 5, 6])
def test_fp8_shapes_match_oracle(shape):
    """FP8 on each tile shape it offers (the row-major kernels): each within
    the FP8 bounds of the oracle at the FP8-rounded J."""
    import paper_1502_04993_amd as G
    from test_gpu_parity import TOL, round_fp8_rows
    rec = synth.balanced(N=512, B=40_000, seed=24)
    J8 = round_fp8_rows(rec.J)
    ref = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, rec.tau, J8, rec.mu)
    old = os.environ.pop("GLMR_RES_SHAPE", None)
    os.environ["GLMR_RES_SHAPE"] = f"{shape},{shape}"
    try:
        ctx = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision="fp8")
    finally:
        os.environ.pop("GLMR_RES_SHAPE", None)
        if old is not None:
            os.environ["GLMR_RES_SHAPE"] = old
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    ctx.set_params(J8, rec.mu)
    r = ctx.eval(grad=True)
    assert ctx.query()["trace_resident"] and not ctx.query()["trace_frag"]
    ctx.close()
    check(f"fp8 shape {shape}", r, ref, TOL["fp8"])


@pytest.mark.parametrize("frag", [True, False])
def test_autotune_picks_valid_shapes_and_caches(tmp_path, frag):
    rec = synth.balanced(N=384, B=30_000, seed=22)  # Np = 384: only the 128-neuron tiles fit
    cache = str(tmp_path / "tune.txt")
    ctx = _ctx(rec, frag=frag)
    ctx.set_params(rec.J, rec.mu)
    u, g = ctx.autotune(cache)
    if frag:
        assert u == 7 and g == 9  # one kernel U; kernel G's 256- and 512-row tiles do not divide 384
    else:
        assert u in (3, 4, 5, 6) and g in (3, 4, 5, 6)
    a = ctx.eval(grad=True)
    ctx.close()
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("glmrec-tune ")
    ctx = _ctx(rec, frag=frag)
    ctx.set_params(rec.J, rec.mu)
    assert ctx.autotune(cache) == (u, g)  # served from the cache
    b = ctx.eval(grad=True)
    ctx.close()
    assert len(open(cache).read().splitlines()) == 1
    assert a["ll"] == b["ll"] and np.array_equal(a["gJ"], b["gJ"])


def test_autotune_is_a_no_op_without_resident_trace():
    rec = synth.balanced(N=64, B=5_000, seed=23)
    import paper_1502_04993_amd as G
    ctx = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision="fp32")
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    ctx.set_params(rec.J, rec.mu)
    assert ctx.autotune() == (-1, -1)
    ctx.close()
