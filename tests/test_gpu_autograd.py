"""Differentiation form: torch.autograd over (J, mu, tau) with the trace
rebuilt in the backward pass; checked against the FP64 oracle gradient and
central finite differences (h = 1e-6, FP64)."""
import numpy as np
import pytest
import torch

import synth
from oracle import glm_oracle as O

pytestmark = pytest.mark.gpu


def _ctx(rec, prec="fp64"):
    import paper_1502_04993_amd as G
    ctx = G.Context(rec.n_neurons, rec.n_bins, rec.dt, precision=prec)
    ctx.set_spikes(rec.bins, rec.neurons)
    return ctx


def _rec():
    # the config-4 generator (N = 500, in-degree 50, true tau 8 ms), 60 s
    return synth.cached("config4", seed=0, B=60_000)


def test_autograd_matches_oracle_and_fd():
    from paper_1502_04993_amd.autograd import log_likelihood
    rec = _rec()
    N = rec.n_neurons
    ctx = _ctx(rec)
    rng = np.random.default_rng(0)
    J0 = rec.J + rng.normal(0, 0.05, (N, N))
    dev = "cuda"
    J = torch.tensor(J0, dtype=torch.float64, device=dev, requires_grad=True)
    mu = torch.tensor(rec.mu, dtype=torch.float64, device=dev, requires_grad=True)
    tau = torch.tensor(0.015, dtype=torch.float64, requires_grad=True)  # tau_init = 15 ms
    L = log_likelihood(ctx, J, mu, tau)
    L.backward()
    gJ, gmu, gtau = J.grad.cpu().numpy(), mu.grad.cpu().numpy(), float(tau.grad)
    ref = O.loglik(rec.bins, rec.neurons, N, rec.n_bins, rec.dt, 0.015, J0, rec.mu, want_tau=True)
    rl = abs(float(L.detach()) - ref["ll"]) / abs(ref["ll"])
    rg = np.linalg.norm(np.concatenate([gmu - ref["gmu"], (gJ - ref["gJ"]).ravel()])) / \
        np.linalg.norm(np.concatenate([ref["gmu"], ref["gJ"].ravel()]))
    rt = abs(gtau - ref["gtau"]) / abs(ref["gtau"])
    print(f"[autograd fp64] rel_ll={rl:.2e} rel_grad={rg:.2e} rel_gtau={rt:.2e}", flush=True)
    assert rl < 1e-12 and rg < 1e-10 and rt < 1e-10

    # central differences of the GPU likelihood, h = 1e-6
    h = 1e-6

    def Lval(Jm, mum, t):
        with torch.no_grad():
            return float(log_likelihood(ctx, Jm, mum, torch.tensor(t, dtype=torch.float64)))

    Jd, mud = J.detach(), mu.detach()
    fd_tau = (Lval(Jd, mud, 0.015 + h) - Lval(Jd, mud, 0.015 - h)) / (2 * h)
    assert abs(fd_tau - gtau) <= 1e-6 * abs(gtau), (fd_tau, gtau)
    idx = rng.integers(0, N, (12, 2))
    for i, j in idx:
        Jp = Jd.clone(); Jp[i, j] += h
        Jm = Jd.clone(); Jm[i, j] -= h
        fd = (Lval(Jp, mud, 0.015) - Lval(Jm, mud, 0.015)) / (2 * h)
        assert abs(fd - gJ[i, j]) <= 1e-5 * (1 + abs(gJ[i, j])), (i, j, fd, gJ[i, j])
    for i in rng.integers(0, N, 4):
        mp = mud.clone(); mp[i] += h
        mm = mud.clone(); mm[i] -= h
        fd = (Lval(Jd, mp, 0.015) - Lval(Jd, mm, 0.015)) / (2 * h)
        assert abs(fd - gmu[i]) <= 1e-5 * (1 + abs(gmu[i]))
    ctx.close()


def test_profile_likelihood_recovers_tau():
    """tau as a learnable parameter: from 15 ms to the generating 8 ms."""
    from paper_1502_04993_amd.autograd import profile_tau
    rec = synth.cached("config4", seed=0, B=600_000)
    ctx = _ctx(rec, "fp32")
    ctx.set_kernel(0.015)
    ctx.fit(max_iter=300, from_zero=True, warm_start_mu=True)
    tau, hist = profile_tau(ctx, 0.015, steps=10, fit_kwargs=dict(max_iter=300))
    for t, ll, gt in hist:
        print(f"  tau={t * 1e3:.4f} ms  L={ll:.6f}  dL/dtau={gt:.4e}", flush=True)
    print(f"[profile tau] {tau * 1e3:.4f} ms (true 8 ms)", flush=True)
    ctx.close()
    assert abs(tau - 0.008) < 0.0005


def test_autograd_follows_tau_changed_outside():
    """A kernel set on the context between two autograd calls (here by
    Context.set_kernel) must not leak into a call at another tau: the forward
    value and all three gradients are those of the requested tau."""
    from paper_1502_04993_amd.autograd import log_likelihood
    rec = _rec()
    N = rec.n_neurons
    ctx = _ctx(rec)
    J0 = rec.J.copy()
    dev = "cuda"
    t1, t2 = 0.012, 0.006
    ref = O.loglik(rec.bins, rec.neurons, N, rec.n_bins, rec.dt, t1, J0, rec.mu, want_tau=True)
    for k in range(2):
        J = torch.tensor(J0, dtype=torch.float64, device=dev, requires_grad=True)
        mu = torch.tensor(rec.mu, dtype=torch.float64, device=dev, requires_grad=True)
        tau = torch.tensor(t1, dtype=torch.float64, requires_grad=True)
        L = log_likelihood(ctx, J, mu, tau)
        ctx.set_kernel(t2)  # changed between the forward and the backward pass
        L.backward()
        rl = abs(float(L.detach()) - ref["ll"]) / abs(ref["ll"])
        gJ, gmu = J.grad.cpu().numpy(), mu.grad.cpu().numpy()
        rg = np.abs(gJ - ref["gJ"]).max() / np.abs(ref["gJ"]).max()
        rm = np.abs(gmu - ref["gmu"]).max() / np.abs(ref["gmu"]).max()
        rt = abs(float(tau.grad) - ref["gtau"]) / abs(ref["gtau"])
        print(f"[autograd tau changed, call {k}] rel_ll={rl:.2e} gJ={rg:.2e} gmu={rm:.2e} gtau={rt:.2e}",
              flush=True)
        assert rl < 1e-12 and rg < 1e-10 and rm < 1e-10 and rt < 1e-10
        ctx.set_kernel(t2)  # and before the next forward pass
    ctx.close()


def test_autograd_config4_full_length():
    """The differentiation form at the configured length (N = 500, 600 s,
    6e5 bins), tau at its initial 15 ms: L, the gradient (element-wise) and
    dL/dtau against the oracle, and dL/dtau and three J entries against
    central differences of the GPU likelihood (h = 1e-6)."""
    from paper_1502_04993_amd.autograd import log_likelihood
    rec = synth.cached("config4", seed=0, B=600_000)
    N = rec.n_neurons
    ctx = _ctx(rec)
    rng = np.random.default_rng(4)
    J0 = rec.J + rng.normal(0, 0.05, (N, N))
    dev = "cuda"
    J = torch.tensor(J0, dtype=torch.float64, device=dev, requires_grad=True)
    mu = torch.tensor(rec.mu, dtype=torch.float64, device=dev, requires_grad=True)
    tau = torch.tensor(0.015, dtype=torch.float64, requires_grad=True)
    L = log_likelihood(ctx, J, mu, tau)
    L.backward()
    gJ, gmu, gtau = J.grad.cpu().numpy(), mu.grad.cpu().numpy(), float(tau.grad)
    ref = O.loglik(rec.bins, rec.neurons, N, rec.n_bins, rec.dt, 0.015, J0, rec.mu, want_tau=True)
    rl = abs(float(L.detach()) - ref["ll"]) / abs(ref["ll"])
    g = np.concatenate([gmu, gJ.ravel()])
    gr = np.concatenate([ref["gmu"], ref["gJ"].ravel()])
    rg = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    rmax = np.abs(g - gr).max() / np.abs(gr).max()
    rt = abs(gtau - ref["gtau"]) / abs(ref["gtau"])
    print(f"[autograd config4 600 s] rel_ll={rl:.2e} rel_grad={rg:.2e} max={rmax:.2e} rel_gtau={rt:.2e}",
          flush=True)
    assert rl < 1e-12 and rg < 1e-10 and rmax < 1e-10 and rt < 1e-10
    h = 1e-6

    def Lval(Jm, mum, t):
        with torch.no_grad():
            return float(log_likelihood(ctx, Jm, mum, torch.tensor(t, dtype=torch.float64)))

    Jd, mud = J.detach(), mu.detach()
    fd_tau = (Lval(Jd, mud, 0.015 + h) - Lval(Jd, mud, 0.015 - h)) / (2 * h)
    assert abs(fd_tau - gtau) <= 1e-6 * abs(gtau), (fd_tau, gtau)
    for i, j in rng.integers(0, N, (3, 2)):
        Jp = Jd.clone(); Jp[i, j] += h
        Jm = Jd.clone(); Jm[i, j] -= h
        fd = (Lval(Jp, mud, 0.015) - Lval(Jm, mud, 0.015)) / (2 * h)
        assert abs(fd - gJ[i, j]) <= 1e-5 * (1 + abs(gJ[i, j])), (i, j, fd, gJ[i, j])
    ctx.close()
