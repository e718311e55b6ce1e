"""Write stored oracle values for the larger parity cases.

Calls only oracle/ (and the seeded input generator).  The HIP path never
writes anything here.

    python tests/golden/make_oracle_refs.py c2      # -> tests/golden/oracle_c2.npz
    python tests/golden/make_oracle_refs.py c3      # -> tests/golden/oracle_c3.npz

c2: o=10, v=60, naux=120, seed 0, all three dipole directions at w = 0.05:
    E_corr, alpha, and right/left sigma products at seeded (t, X).
c3: o=20, v=150, naux=300, seed 0: E_corr, Omega and A X at the seeded
    probe vectors (4096 sampled entries and full norms), and a few entries of
    X A, each computed on its own as X . (A e_k).  At this size the oracle's
    reverse-mode and forward-mode derivatives do not fit this host's memory,
    so A X uses the exact 5-point contour rule (Omega evaluations only) and
    X A is taken entry by entry.
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.response import (Problem, alpha_from, eta, F_times, left_sigma, right_sigma,  # noqa: E402
                             solve_ground, solve_lambda, solve_x, solve_y, xi)
from oracle.derivs import jvp_contour  # noqa: E402
from paper_2503_23144_amd.synth import config_inputs, probe_vectors  # noqa: E402


def sampled_sigmas(P, seed=11):
    """Omega(t), A X and X A at the seeded probe vectors; 4096 sampled
    entries of each, plus their full norms."""
    t, X, idx = probe_vectors(P.lay.n, seed)
    tt, XX = torch.as_tensor(t), torch.as_tensor(X)
    out = dict(sig_seed=np.array(seed), sig_idx=idx)
    for name, val in (("residual", P.omega(tt)), ("right", right_sigma(P, tt, XX)),
                      ("left", left_sigma(P, tt, XX))):
        v = val.resolve_conj().numpy()
        out["sig_" + name] = v[idx]
        out["sig_" + name + "_norm"] = np.array(np.linalg.norm(v))
    return out


def sampled_sigmas_large(P, seed=11, nleft=8):
    """Omega(t) and A X (contour rule) at the probe vectors; X A at nleft
    indices (half singles, half doubles), each as X . (A e_k)."""
    t, X, idx = probe_vectors(P.lay.n, seed)
    tt, XX = torch.as_tensor(t), torch.as_tensor(X)
    out = dict(sig_seed=np.array(seed), sig_idx=idx)
    t0 = time.time()
    for name, fn in (("residual", lambda: P.omega(tt)),
                     ("right", lambda: jvp_contour(lambda x: P.omega(x), tt, XX))):
        v = fn().resolve_conj().numpy()
        out["sig_" + name] = v[idx]
        out["sig_" + name + "_norm"] = np.array(np.linalg.norm(v))
        print(f"{name} done {time.time() - t0:.0f}s", flush=True)
    rng = np.random.default_rng(seed + 1)
    n1 = P.lay.o * P.lay.v
    kidx = np.concatenate([rng.choice(n1, nleft // 2, replace=False),
                           n1 + rng.choice(P.lay.n - n1, nleft - nleft // 2, replace=False)])
    vals = []
    for k in kidx:
        e = torch.zeros(P.lay.n, dtype=torch.complex128)
        e[int(k)] = 1.0
        Ae = jvp_contour(lambda x: P.omega(x), tt, e)
        vals.append(complex(torch.sum(XX * Ae)))
        print(f"left entry {k} done {time.time() - t0:.0f}s", flush=True)
    out["sig_left_idx"] = kidx
    out["sig_left_entries"] = np.array(vals)
    return out


def main(name):
    inp = config_inputs(name)
    omegas = {"c2": [0.05], "c3": []}[name]
    t0 = time.time()
    P = Problem.from_arrays(inp.B, inp.fock, inp.mu, inp.o)
    out = {}
    out.update(sampled_sigmas(P) if omegas else sampled_sigmas_large(P))
    print(f"sigmas done {time.time() - t0:.0f}s", flush=True)
    t, E, it = solve_ground(P, tol=1e-12)
    print(f"T done ({it} it) {time.time() - t0:.0f}s E={complex(E)}", flush=True)
    if not omegas:
        out.update(ecorr=np.array(complex(E)))
        path = os.path.join(HERE, f"oracle_{name}.npz")
        np.savez(path, **out)
        print(f"wrote {path} in {time.time() - t0:.0f}s", flush=True)
        return
    lam, it = solve_lambda(P, t, tol=1e-12)
    print(f"Lambda done ({it} it) {time.time() - t0:.0f}s", flush=True)
    xis = [xi(P, t, c) for c in range(3)]
    etas = [eta(P, t, lam, c) for c in range(3)]
    alpha = []
    for w in omegas:
        Xs, Ys = [], []
        for c in range(3):
            X, itx = solve_x(P, t, xis[c], w, tol=1e-12)
            Y, ity = solve_y(P, t, lam, etas[c] + F_times(P, t, lam, X), w, tol=1e-12)
            Xs.append(X)
            Ys.append(Y)
            print(f"w={w} comp {c}: X {itx} it, Y {ity} it, {time.time() - t0:.0f}s", flush=True)
        alpha.append(alpha_from(xis, etas, Xs, Ys))
    out.update(ecorr=np.array(complex(E)), omegas=np.array(omegas), alpha=np.array(alpha))
    path = os.path.join(HERE, f"oracle_{name}.npz")
    np.savez(path, **out)
    print(f"wrote {path} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["c2"]:
        main(nm)
