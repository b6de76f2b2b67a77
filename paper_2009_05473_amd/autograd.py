"""Reverse-mode differentiation through libsfw's hand-written adjoint kernels.

Two ``torch.autograd.Function`` classes over the C ABI (argument marshalling only):

* ``ForwardModel``: atoms ``[n, 6]`` = (w, mx, my, mz, sigma, d) -> Phi mu, the observation
  model of section 1.1. The backward pass calls ``sfw_forward_vjp``: Phi^T of the incoming
  volume gradient, then the per-atom sums of section 2's analytic derivatives. Atom
  profiles are recomputed per voxel tile in both passes; no per-atom volume is stored.
* ``Criterion``: atoms -> C = 1/2 ||y - Phi mu||^2 + lambda sum w (section 1.2). The forward
  pass calls ``sfw_residual_grad``, which yields the analytic gradient in the same pass;
  the backward pass scales it.

``slide`` drives the nonconvex sliding step (Algorithm 1 step 4, Algorithm 2's final
descent) over all 6N parameters with a torch optimizer through ``Criterion``.
Gradients with respect to y, H or lambda are not provided.
"""
from __future__ import annotations

import torch

from . import _lib


class ForwardModel(torch.autograd.Function):
    """phi = ForwardModel.apply(atoms, H, ws, vol_shape)."""

    @staticmethod
    def forward(ctx, atoms, H, ws, vol_shape):
        a = atoms.detach().contiguous()
        phi = _lib.sfw_forward(ws, H, a, tuple(vol_shape))
        ctx.ws = ws
        ctx.save_for_backward(a, H)
        return phi

    @staticmethod
    def backward(ctx, g):
        if ctx.needs_input_grad[1]:
            raise NotImplementedError("the gradient with respect to H is not provided")
        a, H = ctx.saved_tensors
        grad = _lib.sfw_forward_vjp(ctx.ws, H, g.detach().contiguous().float(), a)
        return grad, None, None, None


class Criterion(torch.autograd.Function):
    """C = Criterion.apply(atoms, y, H, lam, ws): a float64 scalar on the device."""

    @staticmethod
    def forward(ctx, atoms, y, H, lam, ws):
        a = atoms.detach().contiguous()
        _, loss, grad = _lib.sfw_residual_grad(ws, H, y, float(lam), a, want_r=False)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, gC):
        if ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
            raise NotImplementedError("gradients with respect to y and H are not provided")
        (grad,) = ctx.saved_tensors
        return (gC.to(torch.float64) * grad.to(torch.float64)).to(torch.float32), None, None, \
            None, None


def forward_model(atoms, H, ws, vol_shape):
    return ForwardModel.apply(atoms, H, ws, vol_shape)


def criterion(atoms, y, H, lam, ws):
    return Criterion.apply(atoms, y, H, lam, ws)


def slide(ws, y, H, lam, atoms, lower, upper, max_iter=50, lr=1.0):
    """Minimise C over all 6N parameters from ``atoms`` with torch.optim.LBFGS (strong-Wolfe
    line search), projecting onto the box [lower, upper] (rows of 6 bounds, broadcast over
    atoms) after every step. Returns (atoms, list of C at the start of each step). A step
    lowers C before the projection; the projection can raise it where a bound is active."""
    x = atoms.detach().clone().contiguous().requires_grad_(True)
    lo = torch.as_tensor(lower, dtype=torch.float32, device=x.device)
    hi = torch.as_tensor(upper, dtype=torch.float32, device=x.device)
    opt = torch.optim.LBFGS([x], lr=lr, max_iter=1, line_search_fn="strong_wolfe",
                            history_size=20)

    def closure():
        opt.zero_grad()
        c = Criterion.apply(x, y, H, lam, ws)
        c.backward()
        return c

    history = []
    for _ in range(max_iter):
        c = opt.step(closure)
        with torch.no_grad():
            x.copy_(torch.maximum(torch.minimum(x, hi), lo))
        history.append(float(c))
    return x.detach(), history
