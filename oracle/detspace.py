"""Brute-force second quantization in a determinant basis (small systems).

Test infrastructure (oracle): never used by the product path.

Used to pin the CCSD working equations and the whole response chain:

* ``cc_residual_bruteforce``: Omega_mu = <mu| exp(-T) H exp(T) |0> and
  E = <0|exp(-T) H exp(T)|0> - <0|H|0> for arbitrary amplitudes, with
  T1 = sum t_ia a+_a a_i and T2 = 1/4 sum t_ijab a+_a a+_b a_j a_i
  (Section II.A, Eqs. 1-5 and 9-10), by explicit matrices.
* ``fci_polarizability``: the exact sum-over-states linear response
  function (Eq. 18) from full configuration interaction.  For two
  electrons CCSD is exact, so LR-CCSD must reproduce it.

The Hamiltonian is H = sum h_pq a+_p a_q + 1/4 sum <pq||rs> a+_p a+_q a_s a_r
with h = f - sum_i <pi||qi>, so that the Fock matrix of the reference
determinant (spinors 0..o-1 occupied) is f.
"""
from __future__ import annotations

import itertools

import numpy as np


class DetSpace:
    def __init__(self, nmo: int, nelec: int):
        self.nmo, self.nelec = nmo, nelec
        self.dets, self.index = {}, {}
        for N in range(max(0, nelec - 2), nelec + 1):
            d = list(itertools.combinations(range(nmo), N))
            self.dets[N] = d
            self.index[N] = {x: k for k, x in enumerate(d)}
        self._ann = {}

    def dim(self, N=None):
        return len(self.dets[self.nelec if N is None else N])

    def ann(self, p: int, N: int) -> np.ndarray:
        """Matrix of a_p from the N-electron to the (N-1)-electron space.
        The sign is (-1)^(number of occupied spinors before p)."""
        key = (p, N)
        if key not in self._ann:
            M = np.zeros((self.dim(N - 1), self.dim(N)))
            idx = self.index[N - 1]
            for k, d in enumerate(self.dets[N]):
                if p in d:
                    pos = d.index(p)
                    M[idx[d[:pos] + d[pos + 1:]], k] = (-1) ** pos
            self._ann[key] = M
        return self._ann[key]

    def _pairs(self):
        N, n = self.nelec, self.nmo
        A1 = [self.ann(p, N) for p in range(n)]          # N   -> N-1
        A2 = [self.ann(p, N - 1) for p in range(n)]      # N-1 -> N-2
        # C_p C_q : (N-2) -> N ;  A_s A_r : N -> (N-2)
        up = np.array([[A1[p].T @ A2[q].T for q in range(n)] for p in range(n)])
        dn = np.array([[A2[s] @ A1[r] for r in range(n)] for s in range(n)])
        return A1, up, dn

    def hamiltonian(self, h, g) -> np.ndarray:
        """h [n, n], g[p,q,r,s] = <pq||rs>."""
        A1, up, dn = self._pairs()
        H = np.einsum("pq,pab,qbc->ac", h, np.array([a.T for a in A1]), np.array(A1))
        # 1/4 sum g_pqrs (C_p C_q)(A_s A_r)
        M = np.einsum("pqrs,srbc->pqbc", g, dn)
        H = H + 0.25 * np.einsum("pqab,pqbc->ac", up, M)
        return H

    def one_body(self, m) -> np.ndarray:
        A1 = [self.ann(p, self.nelec) for p in range(self.nmo)]
        return np.einsum("pq,pab,qbc->ac", m, np.array([a.T for a in A1]), np.array(A1))

    def ref(self) -> np.ndarray:
        e = np.zeros(self.dim())
        e[self.index[self.nelec][tuple(range(self.nelec))]] = 1.0
        return e


def h_core(fock, g_full, o):
    """h = f - sum_i <pi||qi>."""
    return np.asarray(fock) - np.einsum("piqi->pq", np.asarray(g_full)[:, :o, :, :o])


def cc_residual_bruteforce(t1, t2, fock, g_full, o):
    """Returns (Omega1 [o, v], Omega2 full [o, o, v, v] (antisymmetric, only
    i != j, a != b meaningful), E_corr) from explicit exp(-T) H exp(T)."""
    t1 = np.asarray(t1)
    t2 = np.asarray(t2)
    n = np.asarray(fock).shape[0]
    v = n - o
    S = DetSpace(n, o)
    A1, up, dn = S._pairs()
    H = S.hamiltonian(h_core(fock, g_full, o), g_full)
    occ, vir = range(o), range(o, n)
    T = np.zeros((S.dim(), S.dim()), dtype=np.complex128)
    for i in occ:
        for a in vir:
            T += t1[i, a - o] * (A1[a].T @ A1[i])
    for i in occ:
        for j in occ:
            for a in vir:
                for b in vir:
                    c = t2[i, j, a - o, b - o]
                    if c != 0:
                        T += 0.25 * c * (up[a, b] @ dn[j, i])

    def expm_nil(X):
        E = np.eye(X.shape[0], dtype=np.complex128)
        term = E.copy()
        for k in range(1, 2 * o + 3):
            term = term @ X / k
            E = E + term
        return E

    r = S.ref().astype(np.complex128)
    hb0 = expm_nil(-T) @ (H @ (expm_nil(T) @ r))
    e_ref = r @ H @ r
    om1 = np.zeros((o, v), dtype=np.complex128)
    om2 = np.zeros((o, o, v, v), dtype=np.complex128)
    for i in occ:
        for a in vir:
            phi = A1[a].T @ (A1[i] @ r)
            om1[i, a - o] = phi @ hb0
    for i in occ:
        for j in occ:
            if i == j:
                continue
            for a in vir:
                for b in vir:
                    if a == b:
                        continue
                    phi = up[a, b] @ (dn[j, i] @ r)
                    om2[i, j, a - o, b - o] = phi @ hb0
    ecorr = r @ hb0 - e_ref
    return om1, om2, ecorr


def fci_states(fock, g_full, o):
    n = np.asarray(fock).shape[0]
    S = DetSpace(n, o)
    H = S.hamiltonian(h_core(fock, g_full, o), g_full)
    w, U = np.linalg.eigh(H)
    return S, H, w, U


def fci_polarizability(fock, g_full, mu, o, omegas):
    """alpha_AB(w) = -<<A;B>>_w with the exact sum over states (Eq. 18):
        alpha_AB = sum_k [A_0k B_k0 / (w_k - w) + B_0k A_k0 / (w_k + w)].
    Also returns E_FCI - E_ref."""
    S, H, w, U = fci_states(fock, g_full, o)
    r = S.ref()
    ops = [U.conj().T @ S.one_body(m) @ U for m in mu]
    wk = w[1:] - w[0]
    out = np.zeros((len(omegas), len(mu), len(mu)), dtype=np.complex128)
    for k, om in enumerate(omegas):
        for a in range(len(mu)):
            for b in range(len(mu)):
                A0k, Bk0 = ops[a][0, 1:], ops[b][1:, 0]
                B0k, Ak0 = ops[b][0, 1:], ops[a][1:, 0]
                out[k, a, b] = np.sum(A0k * Bk0 / (wk - om) + B0k * Ak0 / (wk + om))
    e_ref = np.real(r @ H @ r)
    return out, w[0] - e_ref, wk
