"""Derivatives of the (holomorphic, polynomial) CC functions.

Test infrastructure (oracle): never used by the product path.

The CC Jacobian (Section II.A, Eq. 30) is A = dOmega/dt.  Omega is a
polynomial of degree 4 in t with no complex conjugation, hence holomorphic.

* ``jvp_contour``: A v from the discrete Cauchy integral over a circle,
      A v = (1 / (N r)) sum_k F(t + r w^k v) w^{-k},  w = exp(2 pi i / N),
  which is exact (up to rounding) for polynomials of degree < N + 1 with
  N = 5 (Lyness and Moler, SIAM J. Numer. Anal. 4, 202 (1967)).
* ``jvp_fwd``: the same product by forward-mode automatic differentiation.
* ``vjp_T``: the transposed product A^T u (bilinear, no conjugation).
  PyTorch's reverse mode returns J^H g for a holomorphic function, so
  A^T u = conj(J^H conj(u)).
"""
from __future__ import annotations

import cmath

import torch
import torch.autograd.forward_ad as fwAD


def jvp_contour(fn, x, v, npts: int = 5):
    nv = torch.max(torch.abs(v))
    if nv == 0:
        return torch.zeros_like(fn(x))
    r = 1.0 / float(nv)
    acc = None
    for k in range(npts):
        w = cmath.exp(2j * cmath.pi * k / npts)
        y = fn(x + (r * w) * v) * (1.0 / w)
        acc = y if acc is None else acc + y
    return acc / (npts * r)


def jvp_fwd(fn, x, v):
    with fwAD.dual_level():
        dx = fwAD.make_dual(x.detach(), v.detach())
        y = fn(dx)
        return fwAD.unpack_dual(y).tangent.detach().clone()


def vjp_T(fn, x, u):
    """Returns (A^T u) where A = d fn / d x at x."""
    xx = x.detach().clone().requires_grad_(True)
    y = fn(xx)
    (g,) = torch.autograd.grad(y, xx, grad_outputs=torch.conj(u))
    return torch.conj(g).detach()


def grad_T(fn_scalar, x):
    """Holomorphic gradient dE/dx of a complex scalar function."""
    xx = x.detach().clone().requires_grad_(True)
    y = fn_scalar(xx)
    (g,) = torch.autograd.grad(y, xx, grad_outputs=torch.ones_like(y))
    return torch.conj(g).detach()
