"""Parity of the HIP likelihood path against the FP64 oracle (needs an MI355X).

Every comparison asserts four errors (tests/parity_check.py): the total L,
the largest per-row error of L_i, the 2-norm of the gradient error over
(dL/dmu, dL/dJ), and its largest element relative to the largest gradient
element.  Bounds (relative to the oracle at the same parameters; the
parameters are chosen representable in the compute precision, since each mode
evaluates the likelihood of the parameters rounded to it):
  FP64: L 1e-12, L_i 1e-11, gradient 1e-10 (2-norm and element-wise).
  FP32: L 1e-10 at the N = 1000 workloads (the stated target).  U = sum_j
        J_ij x_j is accumulated in FP64 from FP32 operands; the remaining
        error of L comes from rounding x to FP32 (stochastically, so it is
        random in sign) and its relative size falls as 1/sqrt(B N); on the
        tiny cases here (B N ~ 1e5-1e6) the bound is 1e-10 sqrt(2e6/(B N)).
        A row averages B terms instead of B N, so a row's error is about
        sqrt(N) times that, and the largest of N such random errors about
        four times its spread: L_i's bound is 4 sqrt(N) times L's.  The gradient contraction takes the same FP32-rounded
        operands widened to FP64 and accumulates in FP64, so the gradient
        error is the trace rounding alone (measured <= 6e-9): bound 1e-6,
        2-norm and element-wise.
  BF16: L 1e-3, L_i 1e-3, gradient 1e-3 (2-norm, the stated target) and
        element-wise (at theta = 0 and near the truth).
"bf16" runs the resident trace (built once per tau, kept in HBM); "bf16-rc"
rebuilds the trace inside the contractions.
  FP8 (no target is set for it): L 2e-3, L_i 5e-3, gradient 3e-2 (2-norm and
        element-wise), at J rounded to the FP8 representation (per-row
        power-of-two scale, e4m3).  The trace is e4m3 (3 mantissa bits) and
        the weights e5m2 (2 bits), both rounded stochastically, so each
        element carries ~5-10 % unbiased noise that averages over the bins;
        what is left in L is second order (the convexity of exp), measured at
        ~3e-4 for N = 1000.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import glm_oracle as O
from parity_check import check

pytestmark = pytest.mark.gpu

TOL = {"fp64": dict(ll=1e-12, row=1e-11, grad=1e-10, gmax=1e-10),
       "fp32": dict(ll=1e-10, row=1e-10, grad=1e-6, gmax=1e-6),
       "bf16": dict(ll=1e-3, row=1e-3, grad=1e-3, gmax=1e-3),
       "bf16-rc": dict(ll=1e-3, row=1e-3, grad=1e-3, gmax=1e-3),
       "fp8": dict(ll=2e-3, row=5e-3, grad=3e-2, gmax=3e-2)}
ALL = ["fp64", "fp32", "bf16", "bf16-rc", "fp8"]


def ll_tol(prec, rec):
    tl = TOL[prec]["ll"]
    if prec == "fp32":
        tl *= max(1.0, (2e6 / (rec.n_bins * rec.n_neurons)) ** 0.5)
    return tl


def tol_for(prec, rec):
    """The four bounds of a mode for a recording (FP32's L bounds scale with
    the number of terms, see the module docstring)."""
    t = dict(TOL[prec])
    if prec == "fp32":
        t["ll"] = ll_tol(prec, rec)
        t["row"] = 4.0 * t["ll"] * rec.n_neurons ** 0.5
    return t


def _G():
    import paper_1502_04993_amd as G
    return G


def _e4m3(y):
    """Round float32 values to the nearest OCP e4m3 value (ties to even),
    |y| <= 448: 3 mantissa bits, exponents down to 2^-6, subnormal step 2^-9."""
    y = np.asarray(y, np.float64)
    a = np.abs(y)
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -6)))
    step = 2.0 ** (e - 3)
    return np.sign(y) * np.round(a / step) * step


def round_fp8_rows(J):
    """J as the FP8 path represents it: per row, a power-of-two scale
    2^floor(log2(448 / max|J_ij|)), the scaled float32 value rounded to e4m3."""
    J = np.asarray(J, np.float64)
    out = np.zeros_like(J)
    for i in range(J.shape[0]):
        m = np.float32(np.max(np.abs(J[i]))) if J.shape[1] else np.float32(0)
        sc = 1.0
        if m > 0:
            _, e = np.frexp(np.float32(448.0) / m)
            sc = 2.0 ** (int(e) - 1)
        y = (J[i].astype(np.float32) * np.float32(sc)).astype(np.float64)
        out[i] = _e4m3(y) / sc
    return out


def _round(J, prec):
    prec = prec.split("-")[0]
    if prec == "fp8":
        return round_fp8_rows(J)
    if prec == "fp32":
        return J.astype(np.float32).astype(np.float64)
    if prec == "bf16":
        import torch
        return torch.tensor(J).to(torch.bfloat16).to(torch.float64).numpy()
    return J


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _gvec(r):
    return np.concatenate([r["gmu"], r["gJ"].ravel()])


def run_gpu(rec, J, mu, prec, tau=None, want_tau=False, **kw):
    G = _G()
    if prec == "bf16-rc":
        prec = "bf16"
        kw.setdefault("trace", "recompute")
    ctx = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision=prec, **kw)
    ctx.set_spikes_allow_silent(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau if tau is None else tau)
    ctx.set_params(J, mu)
    out = ctx.eval(grad=True, want_tau=want_tau)
    out["query"] = ctx.query()
    ctx.close()
    # BF16 keeps the trace resident unless asked not to (these inputs are small); FP8 always does
    assert out["query"]["trace_resident"] == (prec == "fp8" or
                                              (prec == "bf16" and kw.get("trace", "auto") != "recompute"))
    return out


def report(tag, got, ref, tol):
    """Assert the four element-wise errors of got against the oracle's ref."""
    return check(tag, got, ref, tol)


_REC = {}


def small_rec():
    if "small" not in _REC:
        _REC["small"] = synth.balanced(N=37, B=5000, in_frac=0.2, seed=11)
    return _REC["small"]


def theta_for(rec, prec, scale=0.05, seed=0):
    rng = np.random.default_rng(seed)
    J = rec.J + rng.normal(0, scale, rec.J.shape)
    return _round(J, prec), rec.mu.copy()


@pytest.mark.parametrize("prec", ALL)
def test_parity_small_ragged(prec):
    rec = small_rec()
    J, mu = theta_for(rec, prec)
    ref = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, rec.tau, J, mu)
    got = run_gpu(rec, J, mu, prec)
    report(f"small {prec}", got, ref, tol_for(prec, rec))


@pytest.mark.parametrize("prec", ALL)
def test_parity_at_zero_coupling(prec):
    rec = small_rec()
    N = rec.n_neurons
    J = np.zeros((N, N))
    mu = np.zeros(N)
    ref = O.loglik(rec.bins, rec.neurons, N, rec.n_bins, rec.dt, rec.tau, J, mu)
    got = run_gpu(rec, J, mu, prec)
    report(f"zero {prec}", got, ref, tol_for(prec, rec))


@pytest.mark.parametrize("prec", ALL)
def test_multichunk_multisplit(prec):
    rec = synth.balanced(N=70, B=20_000, seed=5)
    J, mu = theta_for(rec, prec, seed=1)
    ref = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, rec.tau, J, mu)
    got = run_gpu(rec, J, mu, prec, chunk_bins=4096)
    assert got["query"]["chunk_bins"] == 4096
    report(f"chunks {prec}", got, ref, tol_for(prec, rec))


@pytest.mark.parametrize("prec", ALL)
def test_last_chunk_with_partial_split(prec):
    # 70100 bins pad to 70144 = 36864 + 33280: the second chunk's 33280 bins
    # split into 192-bin pieces, so its last split is cut short by the chunk end
    rec = synth.balanced(N=70, B=70_100, seed=8)
    J, mu = theta_for(rec, prec, seed=2)
    ref = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, rec.tau, J, mu)
    got = run_gpu(rec, J, mu, prec, chunk_bins=36864)
    assert got["query"]["chunk_bins"] == 36864
    report(f"last chunk {prec}", got, ref, tol_for(prec, rec))


def test_multiple_spikes_per_bin():
    rng = np.random.default_rng(3)
    N, B = 20, 3000
    S = rng.poisson(0.03, (B, N))
    S[100, 3] = 4
    t, i = np.nonzero(S)
    bins = np.repeat(t, S[t, i]).astype(np.int64)
    neu = np.repeat(i, S[t, i]).astype(np.int32)
    perm = rng.permutation(bins.shape[0])  # any input order
    rec = synth.Recording("multi", N, B, 0.001, 0.01, bins[perm], neu[perm], np.zeros((N, N)),
                          np.full(N, np.log(20.0)), 16, 0)
    J = rng.normal(0, 0.3, (N, N))
    mu = rec.mu
    ref = O.loglik(rec.bins, rec.neurons, N, B, rec.dt, rec.tau, J, mu)
    got = run_gpu(rec, J, mu, "fp64")
    assert got["query"]["planes"] == 4
    report("multi fp64", got, ref, TOL["fp64"])


def test_edges_first_last_bin_and_silent_neuron():
    N, B = 9, 1000
    bins = np.array([0, 0, 999, 500, 998, 3, 700, 1, 999], np.int64)
    neu = np.array([0, 1, 2, 3, 4, 5, 6, 7, 2], np.int32)  # neuron 8 never fires
    rec = synth.Recording("edges", N, B, 0.001, 0.005, bins, neu, np.zeros((N, N)), np.zeros(N), 7, 0)
    rng = np.random.default_rng(0)
    J = rng.normal(0, 0.5, (N, N))
    mu = rng.normal(1.0, 0.2, N)
    G = _G()
    ctx = G.Context(N, B, 0.001, precision="fp64")
    with pytest.raises(G.GlmrError) as e:
        ctx.set_spikes(bins, neu)
    assert e.value.status == -4  # ENOSPIKES, raster kept
    ctx.set_kernel(0.005)
    ctx.set_params(J, mu)
    got = ctx.eval(grad=True)
    with pytest.raises(G.GlmrError):
        ctx.fit(max_iter=2)  # MLE of the silent neuron does not exist
    ctx.close()
    ref = O.loglik(bins, neu, N, B, 0.001, 0.005, J, mu)
    report("edges fp64", got, ref, TOL["fp64"])


def test_rejects_out_of_range_spikes():
    G = _G()
    ctx = G.Context(5, 100, 0.001, precision="fp32")
    with pytest.raises(G.GlmrError) as e:
        ctx.set_spikes(np.array([3, 100], np.int64), np.array([0, 1], np.int32))
    assert e.value.status == -1 and "index 1" in str(e.value)
    with pytest.raises(G.GlmrError):
        ctx.set_spikes(np.array([3], np.int64), np.array([5], np.int32))
    with pytest.raises(G.GlmrError):
        ctx.set_kernel(0.0005)  # tau < dt
    with pytest.raises(G.GlmrError) as e:
        ctx.eval()
    assert e.value.status == -6  # call order
    ctx.close()


def test_empty_raster():
    N, B = 4, 600
    G = _G()
    ctx = G.Context(N, B, 0.001, precision="fp64")
    st = ctx.set_spikes_allow_silent(np.zeros(0, np.int64), np.zeros(0, np.int32))
    assert st == -4
    ctx.set_kernel(0.01)
    mu = np.log(np.array([2.0, 3.0, 4.0, 5.0]))
    ctx.set_params(np.zeros((N, N)), mu)
    got = ctx.eval(grad=True)
    ctx.close()
    # no spikes: L_i = -T e^{mu_i}
    assert np.allclose(got["ll_rows"], -B * 0.001 * np.exp(mu), rtol=1e-14)
    assert np.allclose(got["gJ"], 0.0)


# dL/dtau is a component of the gradient: BF16 takes the gradient's bound
# (measured 1.3e-5 and 1.9e-5)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-6), ("bf16", 1e-3), ("bf16-rc", 1e-3)])
def test_tau_gradient(prec, tol):
    rec = synth.balanced(N=40, B=6000, tau=0.008, seed=8)
    J, mu = theta_for(rec, prec, seed=2)
    tau = 0.012
    ref = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, tau, J, mu, want_tau=True)
    got = run_gpu(rec, J, mu, prec, tau=tau, want_tau=True)
    r = abs(got["gtau"] - ref["gtau"]) / abs(ref["gtau"])
    print(f"[tau {prec}] gtau={got['gtau']:.8e} ref={ref['gtau']:.8e} rel={r:.2e}", flush=True)
    assert r <= tol


@pytest.mark.parametrize("prec", ["bf16", "bf16-rc"])
def test_tau_gradient_many_tiles_and_chunks(prec):
    # N = 300 pads to 384 (three 128-neuron tiles, i0 > 0) and chunk_bins = 4096
    # splits the 30016 padded bins into seven full chunks and a short last one:
    # the tile-major weights that the resident trace's dL/dtau contraction
    # reads are addressed at every tile and chunk offset
    rec = synth.balanced(N=300, B=30_000, tau=0.008, seed=12)
    J, mu = theta_for(rec, prec, seed=5)
    tau = 0.011
    ref = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, tau, J, mu, want_tau=True)
    got = run_gpu(rec, J, mu, prec, tau=tau, want_tau=True, chunk_bins=4096)
    assert got["query"]["chunk_bins"] == 4096 and got["query"]["n_pad"] == 384
    r = abs(got["gtau"] - ref["gtau"]) / abs(ref["gtau"])
    print(f"[tau tiles {prec}] gtau={got['gtau']:.8e} ref={ref['gtau']:.8e} rel={r:.2e}", flush=True)
    report(f"tau tiles {prec}", got, ref, tol_for(prec, rec))
    assert r <= 1e-3


@pytest.mark.parametrize("prec", ["bf16", "bf16-rc", "fp8"])
def test_determinism_bitwise(prec):
    rec = small_rec()
    J, mu = theta_for(rec, prec)
    a = run_gpu(rec, J, mu, prec)
    b = run_gpu(rec, J, mu, prec)
    assert a["ll"] == b["ll"] and np.array_equal(a["gJ"], b["gJ"])


def test_fp8_rejects_tau_gradient_and_rebuilt_trace():
    rec = small_rec()
    G = _G()
    with pytest.raises(G.GlmrError):
        G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision="fp8", trace="recompute")
    ctx = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision="fp8")
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    ctx.set_params(_round(rec.J, "fp8"), rec.mu)
    with pytest.raises(G.GlmrError) as e:
        ctx.eval(grad=True, want_tau=True)
    assert e.value.status == -1
    ctx.close()


def test_config1_fp64():
    rec = synth.config1(0)
    N = rec.n_neurons
    for tag, J, mu in (("zero", np.zeros((N, N)), np.zeros(N)), ("truth", rec.J, rec.mu)):
        ref = O.loglik(rec.bins, rec.neurons, N, rec.n_bins, rec.dt, rec.tau, J, mu)
        got = run_gpu(rec, J, mu, "fp64")
        report(f"config1 {tag}", got, ref, TOL["fp64"])


_BIG = {}


def big_rec():
    """The N = 1000 balanced network of the headline workload, 131 s long
    (131072 bins, two oracle chunks, so the FP64 oracle finishes in seconds)."""
    if "big" not in _BIG:
        _BIG["big"] = synth.config2(0, B=131_072)
    return _BIG["big"]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16-rc", "fp8"])
@pytest.mark.parametrize("where", ["zero", "truth"])
def test_n1000_parity(prec, where):
    rec = big_rec()
    N = rec.n_neurons
    if where == "zero":
        J, mu = np.zeros((N, N)), np.zeros(N)
    else:
        J, mu = _round(rec.J, prec), rec.mu.copy()
    ref = O.loglik(rec.bins, rec.neurons, N, rec.n_bins, rec.dt, rec.tau, J, mu)
    got = run_gpu(rec, J, mu, prec)
    report(f"n1000 {where} {prec}", got, ref, tol_for(prec, rec))


def _bf16_rne(x):
    """Round to BF16 through FP32, both to nearest even (as the library stages J)."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def two_term_j(J):
    """J as GLMR_BF16_J2 represents it: bf16(J) + bf16(J - bf16(J))."""
    hi = _bf16_rne(J)
    return hi + _bf16_rne(J - hi)


@pytest.mark.parametrize("case", ["small", "chunks", "n1000"])
def test_bf16_two_term_j(case):
    """BF16 with J as two BF16 terms: the BF16 bounds against the oracle at the
    two-term value of J, which is within ~1e-5 relative of J itself (so the
    oracle at the unrounded J gives almost the same errors), while BF16's
    one-term J is 4e-3 steps away."""
    G = _G()
    if case == "small":
        rec, kw = small_rec(), {}
    elif case == "chunks":
        rec, kw = synth.balanced(N=70, B=20_000, seed=5), dict(chunk_bins=4096)
    else:
        rec, kw = big_rec(), {}
    rng = np.random.default_rng(9)
    J = rec.J + rng.normal(0, 0.05, rec.J.shape)  # not representable in BF16
    J2 = two_term_j(J)
    assert np.abs(J2 - J).max() <= 2.0 ** -16 * np.abs(J).max()
    ref = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, rec.tau, J2, rec.mu)
    ctx = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision="bf16j2", **kw)
    ctx.set_spikes(rec.bins, rec.neurons)
    ctx.set_kernel(rec.tau)
    ctx.set_params(J, rec.mu)
    got = ctx.eval(grad=True)
    assert ctx.query()["trace_resident"]
    with pytest.raises(G.GlmrError):
        ctx.eval(want_tau=True)
    # switching to one-term BF16 and back keeps the trace; the one-term
    # likelihood is that of bf16(J)
    ctx.set_precision("bf16")
    one = ctx.eval(grad=True)
    ctx.set_precision("bf16j2")
    again = ctx.eval(grad=True)
    ctx.close()
    report(f"two-term J {case}", got, ref, TOL["bf16"])
    assert again["ll"] == got["ll"] and np.array_equal(again["gJ"], got["gJ"])
    ref1 = O.loglik(rec.bins, rec.neurons, rec.n_neurons, rec.n_bins, rec.dt, rec.tau, _bf16_rne(J), rec.mu,
                    want_grad=False)
    report(f"one-term J after the switch {case}", dict(ll=one["ll"], ll_rows=one["ll_rows"]), ref1,
           TOL["bf16"])
