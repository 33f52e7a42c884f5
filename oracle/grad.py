"""FP64 reference gradients of a loss on the JKO flow output.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  This is the reduced
scaling iteration of ``jko_oracle.jko_step`` (Proposition 3.3 with the u, v
corrections dropped) written with torch float64 CPU tensors, unrolled at fixed
iteration counts, and differentiated by torch autograd.  The JKO flow
(eq. smooth-jko) chains the steps with q = p_t, cold-starting each one
(Listing 1, step 2).

Energies: ``zero``, ``congestion`` (Proposition 4.1; the clamp takes the
capped branch on ties), ``entropy`` (Proposition 4.2, m = 1),
``gen_entropy`` (Proposition 4.2 with per-cell weights and exponents): its
prox is the oracle's exact Lambert-W root, differentiated through the
implicit function theorem on eq. prox-psi,
d log psi / d log s = 1 / (1 + sigma b m psi^{m-1}) (psi = D p), and
``porous`` (f = sum c (D p)^m / ((m-1) D)): its prox is the exact Lambert-W
root psi of log psi + k psi^{m-1} = log s, k = sigma c m D^{m-1} / (m-1) (the
first-order condition of the KL prox, as in Proposition 4.2), differentiated
the same way: d psi / d s = psi / (s (1 + (m-1) k psi^{m-1})).
"""
from __future__ import annotations

import numpy as np
import torch

from .jko_oracle import log_prox_gen_entropy, prox_porous


def _centres(n):
    return (torch.arange(n, dtype=torch.float64) + 0.5) / n


def _factor(n, gamma):
    x = _centres(n)
    return torch.exp(-(x[:, None] - x[None, :]) ** 2 / gamma)


def _apply(x, factors):
    y = x
    for ax, K in enumerate(factors):
        y = torch.movedim(torch.tensordot(K, torch.movedim(y, ax, 0), dims=([1], [0])), 0, ax)
    return y


class _GenEntropyProx(torch.autograd.Function):
    """p = Prox^KL_{sigma f}(s) for the generalised entropies (values from the
    exact root; derivatives in s and in the weights b from the implicit
    function theorem on Y + c (e^{eps Y} - 1)/eps = log(D s), c = sigma b m,
    Y = log(D p): dY/dlog s = 1/(1 + c e^{eps Y}),
    dY/db = -sigma m (e^{eps Y} - 1)/eps / (1 + c e^{eps Y}))."""

    @staticmethod
    def forward(ctx, s, sigma, b, m, D):
        with np.errstate(divide="ignore"):
            lp = log_prox_gen_entropy(np.log(s.detach().numpy()), sigma, b.numpy(), m.numpy(), D)
        p = torch.from_numpy(np.exp(lp))
        ctx.save_for_backward(s, p, b, m)
        ctx.sigma, ctx.D = sigma, D
        return p

    @staticmethod
    def backward(ctx, gp):
        s, p, b, m = ctx.saved_tensors
        Y = torch.log(ctx.D * p)
        eps = m - 1.0
        ey = torch.exp(eps * Y)
        dlog = 1.0 / (1.0 + ctx.sigma * b * m * ey)
        ds = torch.where(s > 0, gp * dlog * p / torch.where(s > 0, s, torch.ones_like(s)), torch.zeros_like(s))
        phi = torch.where(eps > 0, torch.expm1(eps * Y) / torch.where(eps > 0, eps, torch.ones_like(eps)), Y)
        db = torch.where(s > 0, -gp * p * ctx.sigma * m * phi * dlog, torch.zeros_like(s))
        return ds, None, db, None, None


class _PorousProx(torch.autograd.Function):
    """p = Prox^KL_{sigma f}(s) for the porous-medium energy: the exact root
    psi of log psi + k psi^{m-1} = log s (values from the oracle's Lambert-W
    form), with the derivative in s from the implicit function theorem on that
    equation, d psi / d s = psi / (s (1 + (m-1) k psi^{m-1})); 0 where s = 0."""

    @staticmethod
    def forward(ctx, s, k, m):
        p = torch.from_numpy(prox_porous(s.detach().numpy(), k.numpy(), m))
        ctx.save_for_backward(s, p, k)
        ctx.m = m
        return p

    @staticmethod
    def backward(ctx, gp):
        s, p, k = ctx.saved_tensors
        m = ctx.m
        pos = s > 0
        dpds = p / (torch.where(pos, s, torch.ones_like(s)) * (1.0 + (m - 1.0) * k * p ** (m - 1.0)))
        return torch.where(pos, gp * dpds, torch.zeros_like(s)), None, None


def flow_torch(p0, w, kappa, gamma, tau, iters_per_step, kind="congestion", coef=None, m=None,
               density_scale=1.0):
    """Differentiable flow output p_T (torch tensors in, torch tensor out)."""
    shape = tuple(p0.shape)
    factors = [_factor(n, gamma) for n in shape]
    sigma = tau / gamma
    q = p0
    for K in iters_per_step:
        a = torch.ones(shape, dtype=torch.float64)
        p = None
        for _ in range(K):
            t = _apply(a, factors)
            b = q / t
            s = _apply(b, factors)
            if kind == "congestion":
                sg = s * torch.exp(-sigma * w)
                p = torch.where(sg < kappa, sg, kappa)
            elif kind == "entropy":
                p = s ** (1.0 / (1.0 + sigma * coef))
            elif kind == "gen_entropy":
                p = _GenEntropyProx.apply(s, sigma, coef, m, density_scale)
            elif kind == "porous":
                # m is the scalar exponent here; k = sigma c m D^{m-1} / (m - 1)
                k = sigma * coef * m * density_scale ** (m - 1.0) / (m - 1.0)
                p = _PorousProx.apply(s, k.detach(), m)
            elif kind == "zero":
                p = s
            else:
                raise ValueError(kind)
            a = p / s
        q = p
    return q


def loss_and_grads(p0, w, kappa, gamma, tau, iters_per_step, target, kind="congestion",
                   coef=None, m=None, density_scale=1.0):
    """loss = ||p_T - target||^2 and its gradients with respect to w and p0,
    all as float64 numpy arrays."""
    tp0 = torch.tensor(np.asarray(p0, np.float64), requires_grad=True)
    tw = torch.tensor(np.asarray(w, np.float64), requires_grad=True)
    tk = torch.tensor(np.broadcast_to(np.asarray(kappa, np.float64), p0.shape).copy())
    tc = None if coef is None else torch.tensor(np.broadcast_to(np.asarray(coef, np.float64), p0.shape).copy(),
                                                requires_grad=(kind == "gen_entropy"))
    if kind == "porous":
        tm = float(m)   # one exponent for the whole grid
    else:
        tm = None if m is None else torch.tensor(np.broadcast_to(np.asarray(m, np.float64), p0.shape).copy())
    pT = flow_torch(tp0, tw, tk, gamma, tau, iters_per_step, kind, tc, tm, density_scale)
    loss = ((pT - torch.tensor(np.asarray(target, np.float64))) ** 2).sum()
    loss.backward()
    # the gradient in the energy's per-cell field: w, or the weights b of the
    # generalised entropies
    gw = tc.grad.numpy().copy() if kind == "gen_entropy" else (None if tw.grad is None else tw.grad.numpy().copy())
    return float(loss.detach()), gw, tp0.grad.numpy().copy(), pT.detach().numpy()
