"""Antisymmetrized complex spinor integrals from density-fitting factors.

Test infrastructure (oracle): never used by the product path.

The paper's correlated equations use antisymmetrized two-electron integrals
<pq||rs> over complex molecular spinors (Section II.B, Eq. 39).  Here the
Coulomb integrals come from density-fitting factors,
    (pr|qs) = sum_Q B^Q_pr B^Q_qs,
and
    <pq||rs> = <pq|rs> - <pq|sr> = (pr|qs) - (ps|qr).
"""
from __future__ import annotations

import torch


def _sl(o: int, c: str) -> slice:
    return slice(0, o) if c == "o" else slice(o, None)


def eri_block(B: torch.Tensor, o: int, spec: str) -> torch.Tensor:
    """<pq||rs> for p, q, r, s restricted to the classes in ``spec``
    (e.g. 'ovvo' gives <mb||ej>, indices m occ, b vir, e vir, j occ)."""
    P, Q, R, S = (_sl(o, c) for c in spec)
    coul = torch.einsum("xpr,xqs->pqrs", B[:, P, R], B[:, Q, S])
    exch = torch.einsum("xps,xqr->pqrs", B[:, P, S], B[:, Q, R])
    return coul - exch


def eri_full(B: torch.Tensor) -> torch.Tensor:
    """All of <pq||rs> (small systems only)."""
    coul = torch.einsum("xpr,xqs->pqrs", B, B)
    return coul - coul.permute(0, 1, 3, 2)


class Blocks:
    """Lazily built, cached integral blocks keyed by class string."""

    def __init__(self, B, o: int):
        self.B = torch.as_tensor(B, dtype=torch.complex128)
        self.o = o
        self._cache: dict[str, torch.Tensor] = {}

    def __call__(self, spec: str) -> torch.Tensor:
        if spec not in self._cache:
            self._cache[spec] = eri_block(self.B, self.o, spec)
        return self._cache[spec]


class ZeroBlocks:
    """The two-electron operator set to zero (used for one-electron
    perturbations: the f-linear part of Omega)."""

    def __init__(self, o: int, v: int):
        self.o, self.v = o, v

    def __call__(self, spec: str) -> torch.Tensor:
        shape = [self.o if c == "o" else self.v for c in spec]
        return torch.zeros(shape, dtype=torch.complex128)
