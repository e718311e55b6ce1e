"""Seeded synthetic inputs shaped like the paper's systems.

This module holds no arithmetic of the method: it only draws random numbers.
Both the FP64 CPU oracle (``oracle/``) and the HIP path consume what it returns.

The paper's workloads are heavy-element atoms and molecules with Dyall basis
sets and four-component Dirac-Hartree-Fock integrals (Section III), which are
not reproducible here.  These inputs stand in for them with the shapes the
paper reports: 60 retained virtual spinors for HI (Computational Efficiency
section), about 250 of 1002 for I2 (Table V discussion), and more than 1200
virtual spinors before truncation (Abstract).

Recipe (fixed draw order, numpy PCG64):
  B^Q_pq   = 0.5 (G + G^H)_pq * 0.05 / sqrt(naux),  G ~ N(0,1) + i N(0,1)
             (Hermitian in pq for every Q; density-fitting factors)
  eps_occ  ~ U[-2.0, -0.3] (sorted),  eps_vir ~ U[0.2, 5.0] (sorted), Hartree
  F        = diag(eps) (complex)
  mu_c     = 0.05 (M + M^H),  M ~ N(0,1) + i N(0,1),  c = x, y, z
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Inputs:
    o: int
    v: int
    naux: int
    B: np.ndarray        # [naux, nmo, nmo] complex128, Hermitian per Q
    fock: np.ndarray     # [nmo, nmo] complex128 Hermitian (diagonal here)
    mu: np.ndarray       # [3, nmo, nmo] complex128 Hermitian
    omegas: np.ndarray   # [nw] float64 (Hartree)
    seed: int

    @property
    def nmo(self) -> int:
        return self.o + self.v

    @property
    def gap(self) -> float:
        e = np.real(np.diag(self.fock))
        return float(e[self.o:].min() - e[:self.o].max())


# Workloads: (o, v, naux, omegas).  The first is the small case the oracle
# finishes in seconds; the rest grow toward the paper's truncated spaces.
CONFIGS = {
    "c1": dict(o=4, v=16, naux=32, omegas=[0.0]),
    "c2": dict(o=10, v=60, naux=120, omegas=[0.05]),
    "c3": dict(o=20, v=150, naux=300, omegas=list(np.linspace(0.0, 0.3, 16))),
    "c4": dict(o=30, v=300, naux=600, omegas=list(np.linspace(0.0, 0.4, 32))),
    "c5": dict(o=40, v=400, naux=800, omegas=list(np.linspace(0.0, 0.5, 64))),
}


def make_inputs(o: int, v: int, naux: int, omegas=(0.0,), seed: int = 0,
                fock_scale: float = 1.0, real: bool = False) -> Inputs:
    """Draw one synthetic system.  ``real=True`` drops the imaginary parts
    (used for the real-orbital special case)."""
    rng = np.random.default_rng(seed)
    nmo = o + v
    G = rng.standard_normal((naux, nmo, nmo)) + 1j * rng.standard_normal((naux, nmo, nmo))
    B = 0.5 * (G + G.conj().transpose(0, 2, 1)) * (0.05 / np.sqrt(naux))
    eps = np.concatenate([np.sort(rng.uniform(-2.0, -0.3, o)),
                          np.sort(rng.uniform(0.2, 5.0, v))]) * fock_scale
    fock = np.diag(eps).astype(np.complex128)
    mus = []
    for _ in range(3):
        M = rng.standard_normal((nmo, nmo)) + 1j * rng.standard_normal((nmo, nmo))
        mus.append(0.05 * (M + M.conj().T))
    mu = np.stack(mus)
    if real:
        B = np.ascontiguousarray(B.real).astype(np.complex128)
        mu = np.ascontiguousarray(mu.real).astype(np.complex128)
    return Inputs(o=o, v=v, naux=naux, B=np.ascontiguousarray(B), fock=fock,
                  mu=np.ascontiguousarray(mu),
                  omegas=np.asarray(omegas, dtype=np.float64), seed=seed)


def make_inputs_on_device(o: int, v: int, naux: int, omegas=(0.0,), seed: int = 0, device="cuda",
                          q_chunk: int = 32) -> Inputs:
    """The same recipe with B drawn on the device (torch's Philox generator,
    seeded, real then imaginary parts per chunk of q_chunk Q), for spaces
    whose host draw would take minutes (naux=800, nmo=1340: 2.9e9 normals).
    eps, F and mu follow make_inputs' distributions from a numpy PCG64
    stream of the same seed.  The values differ from make_inputs'; the
    distributions and the exact Hermiticity of every B^Q are the same.
    ``B`` is returned as a device tensor."""
    import math

    import torch
    rng = np.random.default_rng(seed)
    nmo = o + v
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    B = torch.empty((naux, nmo, nmo), dtype=torch.complex128, device=device)
    for q0 in range(0, naux, q_chunk):
        q1 = min(naux, q0 + q_chunk)
        re = torch.randn((q1 - q0, nmo, nmo), generator=gen, dtype=torch.float64, device=device)
        im = torch.randn((q1 - q0, nmo, nmo), generator=gen, dtype=torch.float64, device=device)
        G = torch.complex(re, im)
        del re, im
        B[q0:q1] = 0.5 * (G + G.conj().transpose(1, 2)) * (0.05 / math.sqrt(naux))
        del G
    eps = np.concatenate([np.sort(rng.uniform(-2.0, -0.3, o)), np.sort(rng.uniform(0.2, 5.0, v))])
    fock = np.diag(eps).astype(np.complex128)
    mus = []
    for _ in range(3):
        M = rng.standard_normal((nmo, nmo)) + 1j * rng.standard_normal((nmo, nmo))
        mus.append(0.05 * (M + M.conj().T))
    return Inputs(o=o, v=v, naux=naux, B=B, fock=fock, mu=np.ascontiguousarray(np.stack(mus)),
                  omegas=np.asarray(omegas, dtype=np.float64), seed=seed)


def config_inputs(name: str, seed: int = 0) -> Inputs:
    c = CONFIGS[name]
    return make_inputs(c["o"], c["v"], c["naux"], c["omegas"], seed=seed)


def random_unitary(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-ish random unitary from the QR of a complex Gaussian matrix."""
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))


def random_vector(n: int, rng: np.random.Generator, scale: float = 1.0) -> np.ndarray:
    return scale * (rng.standard_normal(n) + 1j * rng.standard_normal(n))


def probe_vectors(n: int, seed: int = 11):
    """Seeded (t, X) for spot checks of Jacobian products: t ~ 0.05 N(0,1)
    complex amplitudes, X ~ N(0,1) complex."""
    rng = np.random.default_rng(seed)
    t = 0.05 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    X = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    idx = np.sort(rng.choice(n, size=min(n, 4096), replace=False))
    return t, X, idx
