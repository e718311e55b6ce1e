"""Perturbation-sensitive frozen natural spinors (FNS++), Section II.C.

Test infrastructure (oracle): never used by the product path.

Steps, in the paper's order (Section II.B-II.C, Eqs. 39-50):
 1. MP2 doubles t_ij^ab = <ab||ij> / (e_i + e_j - e_a - e_b)  (Eq. 39; the
    numerator is the conjugate of <ij||ab>, so that E_MP2 = 1/4 sum
    |<ij||ab>|^2 / D is real; this is the first Jacobi step of Omega = 0).
 2. Hbar_ii = F_ii + 1/2 sum t_in^ef <in||ef>,
    Hbar_aa = F_aa - 1/2 sum t_mn^fa <mn||fa>                (Eqs. 49-50).
 3. Per perturbation A (dipole direction):
    Abar_i^a  = A_ai + sum_me A_me t_im^ae        (singles projection of the
                similarity-transformed operator; undefined in Eq. 47),
    Abar_ij^ac = P(a,c) sum_e t_ij^ec A_ae - P(i,j) sum_m t_mj^ac A_mi (Eq. 48),
    t(A)_ij^ac = Abar_ij^ac / (Hbar_aa + Hbar_cc - Hbar_ii - Hbar_jj + s w),
    t(A)_i^a   = Abar_i^a  / (Hbar_aa - Hbar_ii + s w)          (Eqs. 46-47),
    with s = +1 as printed (``omega_sign``).
 4. D^A_ab = 1/2 sum_ijc t(A)_ij^ac conj t(A)_ij^bc + sum_i t(A)_i^a conj t(A)_i^b
    (Eq. 45 read as a Hermitian Gram matrix), averaged over the three
    directions (and over the frequency grid of one batch).
 5. D V = V n (Eq. 41); keep |n| above the threshold (or the top-k).
 6. F~ = V~^H F_vv V~, F~ Z~ = Z~ e~ (Eqs. 42-43); U = V~ Z~ (Eq. 44 read with
    the product order that makes U a (v_full x v_kept) matrix).
 7. Rotate the virtual block of B, mu and f with U.

The ground-state scheme (FNS, Section II.B, Eq. 40) takes steps 5-7 with
the MP2 density D_ab = 1/2 sum_ijc t_ij^ac conj t_ij^bc (same Gram reading)
in place of step 4.
"""
from __future__ import annotations

import numpy as np
import torch

from .integrals import eri_block

einsum = torch.einsum


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.complex128)


def mp2_and_hbar(B, fock, o):
    """MP2 doubles (Eq. 39) and the diagonal Hbar elements (Eqs. 49-50)."""
    B = _t(B)
    f = _t(fock)
    e = torch.real(torch.diagonal(f))
    eo, ev = e[:o], e[o:]
    g_oovv = eri_block(B, o, "oovv")          # <ij||ab>
    g_vvoo = eri_block(B, o, "vvoo")          # <ab||ij>
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    t2 = g_vvoo.permute(2, 3, 0, 1) / d2       # t_ij^ab (MP2)
    Hii = torch.real(torch.diagonal(f)[:o] + 0.5 * einsum("inef,inef->i", t2, g_oovv))
    Haa = torch.real(torch.diagonal(f)[o:] - 0.5 * einsum("mnfa,mnfa->a", t2, g_oovv))
    return t2, Hii, Haa


def perturbed_amplitudes(t2, Hii, Haa, A, o, w, omega_sign=+1.0):
    """First-order t(A)_i^a and t(A)_ij^ac (Eqs. 46-48) for one operator A."""
    A = _t(A)
    A_ai, A_me, A_ae, A_mi = A[o:, :o], A[:o, o:], A[o:, o:], A[:o, :o]
    s1 = A_ai.T + einsum("me,imae->ia", A_me, t2)
    tmp = einsum("ijec,ae->ijac", t2, A_ae)
    s2 = tmp - tmp.transpose(2, 3)
    tmp = einsum("mjac,mi->ijac", t2, A_mi)
    s2 = s2 - (tmp - tmp.transpose(0, 1))
    den1 = Haa[None, :] - Hii[:, None] + omega_sign * w
    den2 = Haa[None, None, :, None] + Haa[None, None, None, :] \
        - Hii[:, None, None, None] - Hii[None, :, None, None] + omega_sign * w
    return s1 / den1, s2 / den2


def fnspp_density(B, fock, mu, o, omegas, omega_sign=+1.0):
    """Direction- and frequency-averaged second-order vv density (Eq. 45)."""
    t2, Hii, Haa = mp2_and_hbar(B, fock, o)
    mu = _t(mu)
    v = Haa.shape[0]
    D = torch.zeros((v, v), dtype=torch.complex128)
    count = 0
    for w in omegas:
        for A in mu:
            tA1, tA2 = perturbed_amplitudes(t2, Hii, Haa, A, o, float(w), omega_sign)
            D = D + 0.5 * einsum("ijac,ijbc->ab", tA2, tA2.conj()) + einsum("ia,ib->ab", tA1, tA1.conj())
            count += 1
    return (D / count).numpy(), t2


def fns_density(B, fock, o):
    """Ground-state MP2 vv density of the FNS scheme (Eq. 40), read as the
    Hermitian Gram matrix D_ab = 1/2 sum_ijc t_ij^ac conj t_ij^bc."""
    t2, _, _ = mp2_and_hbar(B, fock, o)
    return (0.5 * einsum("ijac,ijbc->ab", t2, t2.conj())).numpy(), t2


def fnspp_transform(B, fock, mu, o, omegas, thresh=1e-5, keep=0, omega_sign=+1.0):
    """Returns (U [v_full, v_kept], n (all occupations, sorted by |n| desc),
    new (B, fock, mu) in the truncated semicanonical basis)."""
    D, _ = fnspp_density(B, fock, mu, o, omegas, omega_sign)
    return transform_from_density(D, B, fock, mu, o, thresh, keep)


def fns_transform(B, fock, mu, o, thresh=1e-5, keep=0):
    """The same steps with the ground-state MP2 density (FNS, Eqs. 40-44)."""
    D, _ = fns_density(B, fock, o)
    return transform_from_density(D, B, fock, mu, o, thresh, keep)


def transform_from_density(D, B, fock, mu, o, thresh=1e-5, keep=0):
    """Eqs. 41-44 from a vv density: natural spinors ordered by |n|, the kept
    ones semicanonicalized, and B, fock, mu rotated into that basis."""
    D = 0.5 * (D + D.conj().T)
    n, V = np.linalg.eigh(D)
    order = np.argsort(-np.abs(n), kind="stable")
    n, V = n[order], V[:, order]
    nk = keep if keep > 0 else int(np.sum(np.abs(n) > thresh))
    Vt = V[:, :nk]
    Fvv = np.asarray(fock)[o:, o:]
    Ft = Vt.conj().T @ Fvv @ Vt
    Ft = 0.5 * (Ft + Ft.conj().T)
    et, Z = np.linalg.eigh(Ft)
    U = Vt @ Z
    nmo = np.asarray(fock).shape[0]
    C = np.zeros((nmo, o + nk), dtype=np.complex128)
    C[:o, :o] = np.eye(o)
    C[o:, o:] = U
    Bn = np.einsum("pi,xpq,qj->xij", C.conj(), np.asarray(B), C)
    fn = C.conj().T @ np.asarray(fock) @ C
    mun = np.einsum("pi,xpq,qj->xij", C.conj(), np.asarray(mu), C)
    return U, n, (Bn, fn, mun)


def captured_norm(t1, t2, U):
    """sum_i |t'_i^k|^2 + 1/2 sum_ijc |t'_ij^{kc}|^2 per new virtual k, with the
    first virtual index transformed, t'_ij^{kc} = sum_a t_ij^ac conj(U_ak)."""
    t2 = _t(t2)
    U = _t(U)
    tk = einsum("ijac,ak->ijkc", t2, U.conj())
    out = 0.5 * torch.sum(torch.abs(tk) ** 2, dim=(0, 1, 3))
    if t1 is not None:
        out = out + torch.sum(torch.abs(einsum("ia,ak->ik", _t(t1), U.conj())) ** 2, dim=0)
    return out.numpy()
