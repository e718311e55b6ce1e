"""CCSD residual Omega(t) = <mu| exp(-T) H exp(T) |0> and energy, complex spinors.

Test infrastructure (oracle): never used by the product path.

The paper defines the cluster operator (Section II.A, Eqs. 1-5; T1 carries
coefficient 1, as Eq. 5 with n = 1 gives) and the projected equations
(Eqs. 9-10) but prints no working equations.  The terms below are the
standard spin-orbital CCSD equations (Stanton, Gauss, Watts, Bartlett,
J. Chem. Phys. 94, 4334 (1991)) with two changes for complex spinors: the
singles driver is f_ai and the doubles driver is <ab||ij> (the bra indices of
every integral are the creation indices of H).  The full Fock matrix is used
in F_ae and F_mi (no (1 - delta) split), so Omega is exactly <mu|Hbar|0>
including its diagonal part; Omega is linear in the pair (f, <||>).

These equations are not taken on trust: tests/test_oracle_pins.py checks
Omega and E at arbitrary amplitudes against brute-force determinant-space
exp(-T) H exp(T) (oracle/detspace.py).

Amplitude layout.  A vector x holds the unique amplitudes: x1[i, a] (o*v)
followed by x2[P(i,j), P(a,b)] for i < j, a < b, with the pair index
P(p, q) = q (q - 1) / 2 + p.  Every dot product is over these unique
entries.
"""
from __future__ import annotations

import torch

einsum = torch.einsum


def pair_lists(n: int):
    """(p, q) with p < q in packed order P = q (q-1)/2 + p."""
    p, q = [], []
    for b in range(n):
        for a in range(b):
            p.append(a)
            q.append(b)
    return torch.tensor(p, dtype=torch.long), torch.tensor(q, dtype=torch.long)


class Layout:
    def __init__(self, o: int, v: int):
        self.o, self.v = o, v
        self.O = o * (o - 1) // 2
        self.V = v * (v - 1) // 2
        self.i0, self.i1 = pair_lists(o)
        self.a0, self.a1 = pair_lists(v)
        self.n1 = o * v
        self.n2 = self.O * self.V
        self.n = self.n1 + self.n2

    def split(self, x):
        return x[..., : self.n1].reshape(*x.shape[:-1], self.o, self.v), \
            x[..., self.n1:].reshape(*x.shape[:-1], self.O, self.V)

    def join(self, x1, x2p):
        return torch.cat([x1.reshape(*x1.shape[:-2], -1), x2p.reshape(*x2p.shape[:-2], -1)], dim=-1)

    def unpack(self, x2p):
        """Packed [O, V] -> full antisymmetric [o, o, v, v]."""
        o, v = self.o, self.v
        I0, I1 = self.i0[:, None], self.i1[:, None]
        A0, A1 = self.a0[None, :], self.a1[None, :]
        t = x2p.new_zeros(o, o, v, v)
        t = t.index_put((I0, I1, A0, A1), x2p)
        t = t.index_put((I1, I0, A0, A1), -x2p)
        t = t.index_put((I0, I1, A1, A0), -x2p)
        t = t.index_put((I1, I0, A1, A0), x2p)
        return t

    def pack(self, t):
        """Full [o, o, v, v] -> unique entries [O, V] (i < j, a < b)."""
        return t[self.i0[:, None], self.i1[:, None], self.a0[None, :], self.a1[None, :]]

    def denominators(self, fock) -> torch.Tensor:
        """D_mu = e_a (+ e_b) - e_i (- e_j) from the real Fock diagonal."""
        f = torch.as_tensor(fock, dtype=torch.complex128)
        e = torch.real(torch.diagonal(f)).to(torch.float64)
        eo, ev = e[: self.o], e[self.o:]
        d1 = ev[None, :] - eo[:, None]
        d2 = (ev[self.a0] + ev[self.a1])[None, :] - (eo[self.i0] + eo[self.i1])[:, None]
        return self.join(d1, d2).to(torch.complex128)


def _blocks(f, o):
    return f[:o, :o], f[:o, o:], f[o:, :o], f[o:, o:]


def omega_full(t1, t2, f, g):
    """Residual with full antisymmetric t2.  f: [nmo, nmo] Fock (or any
    one-electron operator), g(spec): antisymmetrized integral blocks.
    Returns (Omega1 [o, v], Omega2 [o, o, v, v])."""
    o = t1.shape[0]
    foo, fov, fvo, fvv = _blocks(f, o)
    tt = einsum("ia,jb->ijab", t1, t1)
    tt = tt - tt.transpose(2, 3)
    tau = t2 + tt
    taut = t2 + 0.5 * tt

    g_oooo, g_ooov, g_oovv = g("oooo"), g("ooov"), g("oovv")
    g_ovvo, g_ovvv, g_vvvv = g("ovvo"), g("ovvv"), g("vvvv")

    # one-particle intermediates
    Fae = fvv - 0.5 * einsum("me,ma->ae", fov, t1) \
        + einsum("mf,mafe->ae", t1, g_ovvv) \
        - 0.5 * einsum("mnaf,mnef->ae", taut, g_oovv)
    Fmi = foo + 0.5 * einsum("ie,me->mi", t1, fov) \
        + einsum("ne,mnie->mi", t1, g_ooov) \
        + 0.5 * einsum("inef,mnef->mi", taut, g_oovv)
    Fme = fov + einsum("nf,mnef->me", t1, g_oovv)

    # two-particle intermediates
    tmp = einsum("je,mnie->mnij", t1, g_ooov)
    Wmnij = g_oooo + tmp - tmp.transpose(2, 3) + 0.25 * einsum("ijef,mnef->mnij", tau, g_oovv)
    # <am||ef> = -<ma||ef>
    tmp = -einsum("mb,maef->abef", t1, g_ovvv)
    Wabef = g_vvvv - tmp + tmp.transpose(0, 1) + 0.25 * einsum("mnab,mnef->abef", tau, g_oovv)
    # <mn||ej> = -<mn||je>
    Wmbej = g_ovvo + einsum("jf,mbef->mbej", t1, g_ovvv) \
        + einsum("nb,mnje->mbej", t1, g_ooov) \
        - einsum("jnfb,mnef->mbej", 0.5 * t2 + einsum("jf,nb->jnfb", t1, t1), g_oovv)

    # singles: <na||if> = -<na||fi>,  <nm||ei> = -<nm||ie>
    r1 = fvo.transpose(0, 1).clone()
    r1 = r1 + einsum("ie,ae->ia", t1, Fae) - einsum("ma,mi->ia", t1, Fmi) \
        + einsum("imae,me->ia", t2, Fme) \
        + einsum("nf,nafi->ia", t1, g_ovvo) \
        - 0.5 * einsum("imef,maef->ia", t2, g_ovvv) \
        + 0.5 * einsum("mnae,nmie->ia", t2, g_ooov)

    # doubles
    r2 = g("vvoo").permute(2, 3, 0, 1).clone()
    Ft = Fae - 0.5 * einsum("mb,me->be", t1, Fme)
    tmp = einsum("ijae,be->ijab", t2, Ft)
    r2 = r2 + tmp - tmp.transpose(2, 3)
    Fmt = Fmi + 0.5 * einsum("je,me->mj", t1, Fme)
    tmp = einsum("imab,mj->ijab", t2, Fmt)
    r2 = r2 - (tmp - tmp.transpose(0, 1))
    r2 = r2 + 0.5 * einsum("mnab,mnij->ijab", tau, Wmnij)
    r2 = r2 + 0.5 * einsum("ijef,abef->ijab", tau, Wabef)
    tmp = einsum("imae,mbej->ijab", t2, Wmbej) \
        - einsum("ie,ma,mbej->ijab", t1, t1, g_ovvo)
    r2 = r2 + tmp - tmp.transpose(0, 1) - tmp.transpose(2, 3) + tmp.permute(1, 0, 3, 2)
    tmp = einsum("ie,abej->ijab", t1, g("vvvo"))
    r2 = r2 + tmp - tmp.transpose(0, 1)
    tmp = einsum("ma,mbij->ijab", t1, g("ovoo"))
    r2 = r2 - (tmp - tmp.transpose(2, 3))
    return r1, r2


def energy_full(t1, t2, f, g):
    """E_CC = sum f_ia t_ia + 1/4 sum <ij||ab> t_ijab + 1/2 sum <ij||ab> t_ia t_jb."""
    o = t1.shape[0]
    fov = f[:o, o:]
    g_oovv = g("oovv")
    return einsum("ia,ia->", fov, t1) + 0.25 * einsum("ijab,ijab->", g_oovv, t2) \
        + 0.5 * einsum("ijab,ia,jb->", g_oovv, t1, t1)


def residual(x, f, g, lay: Layout):
    """Omega on a packed amplitude vector; returns a packed vector."""
    t1, t2p = lay.split(x)
    r1, r2 = omega_full(t1, lay.unpack(t2p), f, g)
    return lay.join(r1, lay.pack(r2))


def energy(x, f, g, lay: Layout):
    t1, t2p = lay.split(x)
    return energy_full(t1, lay.unpack(t2p), f, g)
