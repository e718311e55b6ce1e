"""Ground state, Lambda, first-order response amplitudes and the polarizability.

Test infrastructure (oracle): never used by the product path.

What is computed (Section II.A):
  * T from Omega(t) = 0 (Eq. 10), E_CC from Eq. 9.
  * Lambda from the zeroth-order left equation (Eq. 22 with Eq. 20):
        eta0 + lambda A = 0,  eta0 = dE/dt.
  * X^B(omega) from Eq. 29 with the damping set to zero:
        (A - omega) X = -xi^B,  xi^B = <nu| exp(-T) mu_B exp(T) |0>  (Eq. 31),
    i.e. the part of Omega that is linear in the one-electron operator,
    evaluated with f -> mu_B and <pq||rs> -> 0.
  * Y^B(omega) from Eq. 32:  Y (A + omega) = -(eta^B + F X^B), with
        eta^B = d/dt [E(t; mu_B) + lambda . Omega(t; mu_B)]        (Eq. 33)
        F X   = d/de grad_t L(t + e X),  L = E + lambda . Omega     (Eq. 34).
  * The response function in the form the paper implements (Eq. 35):
        <<A;B>>_w = 1/2 [f_AB(w) + conj f_BA(w)],
        f_AB(w)  = Y^B(w) . xi^A + eta^A . X^B(w)   (bilinear, no conj),
    where the operator P(A,B) swaps A and B and conjugates, and
        alpha_AB(w) = -<<A;B>>_w.
  * Eq. 36 (X(w), X(-w) and the quadratic F term) as a cross-check.

Linear and nonlinear equations are solved by Jacobi steps with the orbital
energy denominators plus DIIS, to tight tolerances; the solution is unique
(away from poles), so the iteration choice does not affect the result.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from .ccsd import Layout, energy, residual
from .derivs import grad_T, jvp_contour, jvp_fwd, vjp_T
from .integrals import Blocks, ZeroBlocks


def _c(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.complex128)


def bdot(a, b):
    """Bilinear dot product over unique amplitudes (no conjugation)."""
    return torch.sum(a * b)


class NoConvergence(RuntimeError):
    pass


def diis_jacobi(resid_fn, x0, denom, tol, ref, maxit=300, ndiis=8):
    """Solve R(x) = 0 with x <- x - R/denom and DIIS extrapolation.
    Converged when ||R|| <= tol * ref.  Returns (x, iterations, ||R||)."""
    x = x0.clone()
    xs, es = [], []
    rn = float("inf")
    for it in range(maxit):
        R = resid_fn(x)
        rn = float(torch.linalg.vector_norm(R))
        if rn <= tol * ref:
            return x, it, rn
        xn = x - R / denom
        xs.append(xn)
        es.append(xn - x)
        if len(xs) > ndiis:
            xs.pop(0)
            es.pop(0)
        m = len(xs)
        if m >= 2:
            Bm = np.zeros((m + 1, m + 1), dtype=np.complex128)
            E = torch.stack(es)
            G = (torch.conj(E) @ E.T).numpy()
            Bm[:m, :m] = G / np.max(np.abs(np.diag(G)))   # scale-free Gram matrix
            Bm[m, :m] = 1.0
            Bm[:m, m] = 1.0
            rhs = np.zeros(m + 1, dtype=np.complex128)
            rhs[m] = 1.0
            c = np.linalg.lstsq(Bm, rhs, rcond=None)[0][:m]
            x = sum(complex(ck) * xk for ck, xk in zip(c, xs))
        else:
            x = xn
    raise NoConvergence(f"no convergence after {maxit} iterations, |R| = {rn:.3e}")


@dataclasses.dataclass
class Problem:
    """Everything the oracle needs about one system."""
    o: int
    v: int
    fock: torch.Tensor
    g: object           # Blocks or ZeroBlocks
    mu: torch.Tensor    # [ncomp, nmo, nmo]
    lay: Layout
    D: torch.Tensor

    @classmethod
    def from_arrays(cls, B, fock, mu, o):
        fock = _c(fock)
        mu = _c(mu)
        v = fock.shape[0] - o
        lay = Layout(o, v)
        return cls(o=o, v=v, fock=fock, g=Blocks(B, o), mu=mu, lay=lay,
                   D=lay.denominators(fock))

    def omega(self, x, f=None, g=None):
        return residual(x, self.fock if f is None else f, self.g if g is None else g, self.lay)

    def energy(self, x, f=None, g=None):
        return energy(x, self.fock if f is None else f, self.g if g is None else g, self.lay)

    def zero(self):
        return torch.zeros(self.lay.n, dtype=torch.complex128)


def solve_ground(P: Problem, tol=1e-13, maxit=300):
    """Returns (t, E_corr, iterations).  Starts from t = 0, so the first
    Jacobi step gives the MP2 amplitudes."""
    R0 = P.omega(P.zero())
    ref = max(float(torch.linalg.vector_norm(R0)), 1e-300)
    t, it, _ = diis_jacobi(lambda x: P.omega(x), P.zero(), P.D, tol, ref, maxit)
    return t, P.energy(t), it


def eta0(P: Problem, t):
    return grad_T(lambda x: P.energy(x), t)


def left_sigma(P: Problem, t, lam, f=None, g=None):
    """lambda A  (= A^T lambda)."""
    return vjp_T(lambda x: P.omega(x, f, g), t, lam)


def right_sigma(P: Problem, t, X, f=None, g=None, exact_contour=False):
    """A X."""
    fn = lambda x: P.omega(x, f, g)
    return jvp_contour(fn, t, X) if exact_contour else jvp_fwd(fn, t, X)


def solve_lambda(P: Problem, t, tol=1e-13, maxit=300):
    e0 = eta0(P, t)
    ref = max(float(torch.linalg.vector_norm(e0)), 1e-300)
    lam, it, _ = diis_jacobi(lambda l: e0 + left_sigma(P, t, l), P.zero(), P.D, tol, ref, maxit)
    return lam, it


def xi(P: Problem, t, comp):
    """xi^B: the one-electron part of Omega with f -> mu_B (Eq. 31)."""
    return P.omega(t, P.mu[comp], ZeroBlocks(P.o, P.v))


def eta(P: Problem, t, lam, comp):
    """eta^B = d/dt [E(t; mu_B) + lambda . Omega(t; mu_B)] (Eq. 33)."""
    Z = ZeroBlocks(P.o, P.v)
    mu = P.mu[comp]
    return grad_T(lambda x: P.energy(x, mu, Z) + bdot(lam, P.omega(x, mu, Z)), t)


def grad_L(P: Problem, x, lam):
    return grad_T(lambda z: P.energy(z) + bdot(lam, P.omega(z)), x)


def F_times(P: Problem, t, lam, X):
    """F X = d/de grad_t L(t + e X) (Eq. 34); grad L is cubic in t, so the
    5-point contour rule is exact."""
    return jvp_contour(lambda x: grad_L(P, x, lam), t, X)


def solve_x(P: Problem, t, xiB, w, tol=1e-13, maxit=300):
    ref = max(float(torch.linalg.vector_norm(xiB)), 1e-300)
    X0 = -xiB / (P.D - w)
    X, it, _ = diis_jacobi(lambda X: right_sigma(P, t, X) - w * X + xiB, X0, P.D - w, tol, ref, maxit)
    return X, it


def solve_y(P: Problem, t, lam, rhs, w, tol=1e-13, maxit=300):
    """rhs = eta^B + F X^B."""
    ref = max(float(torch.linalg.vector_norm(rhs)), 1e-300)
    Y0 = -rhs / (P.D + w)
    Y, it, _ = diis_jacobi(lambda Y: left_sigma(P, t, Y) + w * Y + rhs, Y0, P.D + w, tol, ref, maxit)
    return Y, it


def response_f(xis, etas, Xs, Ys):
    """f_AB = Y^B . xi^A + eta^A . X^B (the unsymmetrized bracket of Eq. 35)."""
    n = len(xis)
    fAB = np.zeros((n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(n):
            fAB[a, b] = complex(bdot(Ys[b], xis[a]) + bdot(etas[a], Xs[b]))
    return fAB


def alpha_from(xis, etas, Xs, Ys):
    """alpha_AB = -1/2 [f_AB + conj f_BA] (Eq. 35 with P(A,B) conjugating)."""
    fAB = response_f(xis, etas, Xs, Ys)
    return -0.5 * (fAB + fAB.T.conj())


@dataclasses.dataclass
class Result:
    ecorr: complex
    t: torch.Tensor
    lam: torch.Tensor
    xi: list
    eta: list
    X: dict
    Y: dict
    FX: dict
    alpha: np.ndarray      # [nw, ncomp, ncomp] complex
    fab: np.ndarray        # [nw, ncomp, ncomp] unsymmetrized f_AB
    iters: dict


def lr_ccsd(B, fock, mu, o, omegas, comps=(0, 1, 2), tol=1e-13) -> Result:
    """Full oracle: T, Lambda, xi, eta, then X, F X, Y and alpha per omega."""
    P = Problem.from_arrays(B, fock, mu, o)
    t, E, it_t = solve_ground(P, tol)
    lam, it_l = solve_lambda(P, t, tol)
    xis = [xi(P, t, c) for c in comps]
    etas = [eta(P, t, lam, c) for c in comps]
    Xs, Ys, FXs, iters = {}, {}, {}, {"t": it_t, "lambda": it_l}
    alpha = np.zeros((len(omegas), len(comps), len(comps)), dtype=np.complex128)
    fab = np.zeros_like(alpha)
    for k, w in enumerate(omegas):
        w = float(w)
        xk, yk = [], []
        for n, c in enumerate(comps):
            X, itx = solve_x(P, t, xis[n], w, tol)
            FX = F_times(P, t, lam, X)
            Y, ity = solve_y(P, t, lam, etas[n] + FX, w, tol)
            Xs[(k, c)], Ys[(k, c)], FXs[(k, c)] = X, Y, FX
            iters[("x", k, c)], iters[("y", k, c)] = itx, ity
            xk.append(X)
            yk.append(Y)
        fab[k] = response_f(xis, etas, xk, yk)
        alpha[k] = -0.5 * (fab[k] + fab[k].T.conj())
    return Result(ecorr=complex(E), t=t, lam=lam, xi=xis, eta=etas, X=Xs, Y=Ys, FX=FXs,
                  alpha=alpha, fab=fab, iters=iters)


def alpha_eq36_from(etas, Xp, Xm, FXp, FXm=None):
    """alpha = -<<A;B>>_w by Eq. 36 from eta^A, X^A(w), X^A(-w) and F X^A(w)
    (and F X^A(-w); when omitted, F is used as symmetric: u.F v = v.F u)."""
    n = len(etas)

    def f36(Xa_m, Xb_p, FXb_p, a, b):
        return complex(bdot(etas[a], Xb_p) + bdot(etas[b], Xa_m) + bdot(Xa_m, FXb_p))

    out = np.zeros((n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(n):
            fp = f36(Xm[a], Xp[b], FXp[b], a, b)      # f(w)
            if FXm is not None:
                fm = f36(Xp[a], Xm[b], FXm[b], a, b)  # f(-w)
            else:
                fm = complex(bdot(etas[a], Xm[b]) + bdot(etas[b], Xp[a]) + bdot(Xm[b], FXp[a]))
            out[a, b] = -0.5 * (fp + np.conj(fm))
    return out


def alpha_eq36(P: Problem, t, lam, comps, w, tol=1e-13):
    """Eq. 36: <<A;B>>_w = 1/2 C^{+-w} P[A(-w), B(w)] (eta^A X^B(w)
    + 1/2 X^A(-w) F X^B(w)); returns alpha = -<<A;B>>."""
    xis = [xi(P, t, c) for c in comps]
    etas = [eta(P, t, lam, c) for c in comps]
    Xp = [solve_x(P, t, x, w, tol)[0] for x in xis]
    Xm = [solve_x(P, t, x, -w, tol)[0] for x in xis]
    FXp = [F_times(P, t, lam, X) for X in Xp]
    FXm = [F_times(P, t, lam, X) for X in Xm]
    return alpha_eq36_from(etas, Xp, Xm, FXp, FXm)


def alpha_uncoupled(fock, mu, o, w):
    """Independent-particle (g = 0, t = 0) limit: sum over single
    excitations, a textbook sum-over-states form (Eq. 18 with
    determinant excitations)."""
    e = np.real(np.diag(fock))
    mu = np.asarray(mu)
    n = mu.shape[0]
    out = np.zeros((n, n), dtype=np.complex128)
    D = e[o:][None, :] - e[:o][:, None]          # [i, a]
    for A in range(n):
        for B in range(n):
            mA_ia = mu[A][:o, o:]
            mB_ai = mu[B][o:, :o].T
            mB_ia = mu[B][:o, o:]
            mA_ai = mu[A][o:, :o].T
            out[A, B] = np.sum(mA_ia * mB_ai / (D - w) + mB_ia * mA_ai / (D + w))
    return out


def alpha_iso(alpha):
    """Isotropic polarizability Tr(alpha)/3 (for a linear molecule this is
    (2 alpha_perp + alpha_par)/3, the convention of Tables IV-VI)."""
    return np.real(np.trace(np.asarray(alpha), axis1=-2, axis2=-1)) / 3.0
