"""Static alpha_zz at o=20, v=150 by finite-field CCSD energies (pin P4 at
the size of the o=20, v=150 workload), written by the oracle alone.

The polarizability is minus the second derivative of the correlation
energy in the field strength (orbital-unrelaxed: f -> f + h mu_z).  Central
differences at h and h/2 with one Richardson step:
    d(h)  = (E(h) - 2 E(0) + E(-h)) / h^2,
    alpha = -Re[d(h/2) + (d(h/2) - d(h)) / 3].
Each field's CCSD equations are solved by the oracle's DIIS-accelerated
Jacobi iteration, started from the zero-field amplitudes, to a residual of
1e-12 relative to the zero-field driving term.  The energies need only the
residual Omega(t), so the whole computation fits this host.

    python tests/golden/make_finite_field_c3.py   # -> tests/golden/oracle_c3_ff.npz
"""
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.response import Problem, diis_jacobi  # noqa: E402
from paper_2503_23144_amd.synth import config_inputs  # noqa: E402

H = 1e-3
TOL = 1e-12


def main():
    inp = config_inputs("c3")
    t0 = time.time()
    P0 = Problem.from_arrays(inp.B, inp.fock, inp.mu, inp.o)
    ref = float(torch.linalg.vector_norm(P0.omega(P0.zero())))
    print(f"reference norm {ref:.6e} ({time.time() - t0:.0f}s)", flush=True)
    tz, it, _ = diis_jacobi(lambda x: P0.omega(x), P0.zero(), P0.D, TOL, ref, 300)
    E0 = complex(P0.energy(tz))
    print(f"E(0) = {E0!r} ({it} it, {time.time() - t0:.0f}s)", flush=True)
    E = {0.0: E0}
    for h in (H, -H, H / 2, -H / 2):
        P = Problem.from_arrays(inp.B, inp.fock + h * inp.mu[2], inp.mu, inp.o)
        t, it, _ = diis_jacobi(lambda x: P.omega(x), tz, P.D, TOL, ref, 300)
        E[h] = complex(P.energy(t))
        print(f"E({h:+.1e}) = {E[h]!r} ({it} it, {time.time() - t0:.0f}s)", flush=True)
    d = lambda h: (E[h] - 2 * E[0.0] + E[-h]) / h ** 2
    alpha = -np.real(d(H / 2) + (d(H / 2) - d(H)) / 3)
    path = os.path.join(HERE, "oracle_c3_ff.npz")
    np.savez(path, alpha_zz_static=np.array(alpha), h=np.array(H), tol=np.array(TOL),
             fields=np.array(sorted(E)), energies=np.array([E[k] for k in sorted(E)]),
             richardson_step=np.array(-np.real(d(H / 2) - d(H)) / 3))
    print(f"alpha_zz(0) = {alpha!r}; wrote {path} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
