"""MP2-level energy and polarizability behind the FNS++ corrections
(Section II.C, Eqs. 51-54).

Test infrastructure (oracle): never used by the product path.

The paper defines the corrections as differences between the full
(canonical) and the truncated virtual space,
    Delta E_MP2 = E_MP2(canonical) - E_MP2(truncated)           (Eqs. 51-52)
    Delta alpha_MP2 = alpha_MP2(canonical) - alpha_MP2(truncated) (Eqs. 53-54),
and says only that the MP2-level polarizability is the linear response
function built from the MP2 amplitudes and the perturbed amplitudes of
Eqs. 46-47.  Reading taken here (both the oracle and the GPU path):
  * t(1) = -Omega(0) / D: the first Jacobi step of the T equations from
    t = 0 (Eq. 39 when the Fock matrix is diagonal); E_MP2 = E(t(1)).
  * lambda(1) = -eta0(0) / D: the first Jacobi step of the Lambda equations
    from lambda = 0, with eta0 = dE/dt at t = 0.
  * X^B(w) = -xi^B / (Dbar - w), with xi^B evaluated at t(1) (at t1 = 0 it
    is the Abar^B of Eqs. 47-48) and Dbar the denominators of Eqs. 46-47
    built from the Hbar diagonals of Eqs. 49-50: the Jacobian of Eq. 29
    replaced by that diagonal, as Eqs. 46-47 do.
  * alpha_MP2 from Eq. 36 at (t(1), lambda(1)) with these X^B(+w), X^B(-w).
"""
from __future__ import annotations

import numpy as np
import torch

from .fnspp import mp2_and_hbar
from .response import Problem, alpha_eq36_from, eta, eta0, F_times, xi


def hbar_denominators(P: Problem, B, fock):
    """Dbar_mu = Hbar_aa (+ Hbar_bb) - Hbar_ii (- Hbar_jj), packed like D."""
    _, Hii, Haa = mp2_and_hbar(B, fock, P.o)
    return P.lay.denominators(torch.diag(torch.cat([Hii, Haa]).to(torch.complex128)))


def mp2_level(B, fock, mu, o, omegas, comps=(0, 1, 2)):
    """Returns (E_MP2, alpha_MP2 [nw, n, n]) under the reading above."""
    P = Problem.from_arrays(B, fock, mu, o)
    z = P.zero()
    t1 = -P.omega(z) / P.D
    lam1 = -eta0(P, z) / P.D
    E = complex(P.energy(t1))
    Dbar = hbar_denominators(P, B, fock)
    xis = [xi(P, t1, c) for c in comps]
    etas = [eta(P, t1, lam1, c) for c in comps]
    alpha = np.zeros((len(omegas), len(comps), len(comps)), dtype=np.complex128)
    for k, w in enumerate(omegas):
        Xp = [-x / (Dbar - w) for x in xis]
        Xm = [-x / (Dbar + w) for x in xis]
        FXp = [F_times(P, t1, lam1, X) for X in Xp]
        alpha[k] = alpha_eq36_from(etas, Xp, Xm, FXp)
    return E, alpha


def first_order(B, fock, mu, o):
    """(t(1), lambda(1), Problem): the first Jacobi steps of T and Lambda."""
    P = Problem.from_arrays(B, fock, mu, o)
    z = P.zero()
    return -P.omega(z) / P.D, -eta0(P, z) / P.D, P
