"""torch.autograd interface to the likelihood (differentiation form).

`LogLikelihood.apply(J, mu, tau, ctx)` returns L(J, mu, tau) as a 0-d float64
tensor.  The forward pass evaluates L only; the backward pass calls the
library again with gradients requested, so the trace x and its
tau-derivative y are rebuilt from the spike times inside the kernels (nothing
from the forward pass is kept but the parameters).  The time constant is not
part of theta_i and L is not concave in it (Sec. 2.2), but it is
differentiable: dL/dtau comes from the extra contraction with y = dx/dtau.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Context, glmr_eval, glmr_get_params


def _as_param(t: torch.Tensor) -> torch.Tensor:
    return t.detach().to(torch.float64).contiguous()


def _sync(ctx: Context, J: torch.Tensor, mu: torch.Tensor, tau: torch.Tensor):
    """Bring the context to (J, mu, tau).  The library's own tau is compared,
    so a kernel set elsewhere (Context.set_kernel, set_state, the
    cross-validation scans) is never mistaken for the requested one; the
    per-tau caches are rebuilt only when the two differ."""
    tv = float(tau.detach().cpu())
    if glmr_get_params(ctx.handle) != tv:
        ctx.set_kernel(tv)
    ctx.set_params(_as_param(J), _as_param(mu))


class LogLikelihood(torch.autograd.Function):
    @staticmethod
    def forward(fctx, J, mu, tau, ctx):
        _sync(ctx, J, mu, tau)
        ll, _ = glmr_eval(ctx.handle)
        fctx.save_for_backward(J, mu, tau)
        fctx.glm = ctx
        return torch.tensor(ll, dtype=torch.float64, device=J.device)

    @staticmethod
    def backward(fctx, g):
        J, mu, tau = fctx.saved_tensors
        ctx = fctx.glm
        _sync(ctx, J, mu, tau)
        dev = J.device
        gJ = torch.empty(J.shape, dtype=torch.float64, device=dev)
        gmu = torch.empty(mu.shape, dtype=torch.float64, device=dev)
        want_tau = bool(fctx.needs_input_grad[2])
        _, gt = glmr_eval(ctx.handle, None, gJ, gmu, want_tau=want_tau)
        gJ = (g * gJ).to(J.dtype) if fctx.needs_input_grad[0] else None
        gmu = (g * gmu).to(mu.dtype) if fctx.needs_input_grad[1] else None
        gtau = (g * torch.tensor(gt, dtype=torch.float64, device=tau.device)).to(tau.dtype) \
            if want_tau else None
        return gJ, gmu, gtau, None


def log_likelihood(ctx: Context, J: torch.Tensor, mu: torch.Tensor, tau: torch.Tensor) -> torch.Tensor:
    """L(J, mu, tau) with gradients to all three (J[i, j] is j -> i)."""
    return LogLikelihood.apply(J, mu, tau, ctx)


def profile_tau(ctx: Context, tau0: float, steps: int = 8, fit_kwargs=None, tau_min=None,
                tau_max=None, tol: float = 1e-5):
    """Maximise the profile likelihood L(theta*(tau), tau) over tau.

    At the inner optimum dL/dtheta = 0, so d/dtau L(theta*(tau), tau) equals the
    partial derivative dL/dtau returned by the backward pass.  The outer
    iteration is a safeguarded secant search on that derivative in log(tau);
    each step refits theta warm-started from the previous optimum.
    Returns (tau, history) with history a list of (tau, L, dL/dtau)."""
    fit_kwargs = dict(fit_kwargs or {})
    dt = ctx.dt
    tau_min = tau_min if tau_min is not None else 1.0001 * dt
    tau_max = tau_max if tau_max is not None else 1e3 * tau0
    hist = []

    def at(tau):
        ctx.set_kernel(tau)
        ctx.fit(**fit_kwargs)
        ll, gt = glmr_eval(ctx.handle, want_tau=True)
        hist.append((tau, ll, gt))
        return ll, gt * tau  # derivative in log(tau)

    u0 = np.log(tau0)
    l0, d0 = at(tau0)
    u1 = u0 + (0.1 if d0 > 0 else -0.1)
    for _ in range(steps):
        u1 = float(np.clip(u1, np.log(tau_min), np.log(tau_max)))
        l1, d1 = at(float(np.exp(u1)))
        if abs(u1 - u0) < tol:
            break
        if d1 != d0:
            u2 = u1 - d1 * (u1 - u0) / (d1 - d0)
        else:
            u2 = u1 + (0.1 if d1 > 0 else -0.1)
        # keep the step bounded (the profile is not concave in tau)
        u2 = u1 + float(np.clip(u2 - u1, -0.5, 0.5))
        u0, d0, u1 = u1, d1, u2
    best = max(hist, key=lambda h: h[1])
    ctx.set_kernel(best[0])
    return best[0], hist
