"""The lean memory layout against the oracle, through the C ABI.

LRCC_MEMORY_LEAN keeps <ov||vv> only packed over its last pair and forms the
dense <ov||vv>, <vv||vo> and <vv||oo> blocks each contraction reads on the
fly, in chunks over their occupied index; mixed precision can keep a single
W (FP32) with the FP64 ladder rebuilt from the factors.  Small chunk sizes
(LRCC_VIRTUAL_CHUNK_BYTES) force the chunked paths at test sizes: contracted
chunks (split K, accumulated), output chunks (a mapped epilogue writing
disjoint parts) and the copy into a primal intermediate.
"""
import os

import numpy as np
import pytest
import torch

from paper_2503_23144_amd.synth import make_inputs

pytestmark = pytest.mark.gpu


def _lrcc():
    from paper_2503_23144_amd import lrcc
    return lrcc


def _rand(rng, *shape, scale=1.0):
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def _relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _ctx(inp, precision="fp64", tol=1e-11, **kw):
    c = _lrcc().Context(precision=precision, tol=tol, **kw)
    c.load_df(inp.o, inp.v, inp.B)
    c.load_fock(inp.fock)
    c.load_dipoles(inp.mu)
    return c


CASES = [("c1", 4, 16, 32, 8.0, 0), ("ragged", 3, 17, 11, 8.0, 5)]


@pytest.mark.parametrize("chunk", [None, 256])
@pytest.mark.parametrize("name,o,v,naux,scale,seed", CASES)
def test_lean_layout_matches_oracle(monkeypatch, name, o, v, naux, scale, seed, chunk):
    from oracle.response import Problem, left_sigma, lr_ccsd, right_sigma
    if chunk is not None:  # one occupied index per chunk
        monkeypatch.setenv("LRCC_VIRTUAL_CHUNK_BYTES", str(chunk))
    print(f"lean layout {name} chunk={chunk}", flush=True)
    inp = make_inputs(o, v, naux, seed=seed)
    inp.B = inp.B * scale
    P = Problem.from_arrays(inp.B, inp.fock, inp.mu, inp.o)
    rng = np.random.default_rng(seed + 17)
    t = _rand(rng, P.lay.n, scale=0.05)
    c = _ctx(inp, memory="lean")
    assert _relerr(c.sigma("residual", t), P.omega(torch.as_tensor(t)).numpy()) < 1e-12
    c.set_amplitudes(_lrcc().AMP_T, t)
    X = _rand(rng, 3, P.lay.n)
    for side, fn in (("right", right_sigma), ("left", left_sigma)):
        got = c.sigma(side, X)
        got32 = c.sigma(side, X, precision="mixed")
        for r in range(3):
            ref = fn(P, torch.as_tensor(t), torch.as_tensor(X[r])).resolve_conj().numpy()
            assert _relerr(got[r], ref) < 1e-12, (side, r)
            assert _relerr(got32[r], ref) < 1e-5, (side, r)
    c.close()
    omegas = [0.0, 0.11]
    ref = lr_ccsd(inp.B, inp.fock, inp.mu, o, omegas, tol=1e-13)
    for prec, ladder, l64, tol in (("fp64", "full", None, 1e-8), ("mixed", "full", "direct", 1e-6),
                                   ("mixed", "triangle", "direct", 1e-6)):
        c = _ctx(inp, precision=prec, tol=1e-11 if prec == "fp64" else 1e-10, memory="lean", ladder=ladder,
                 ladder_fp64=l64)
        e, _ = c.solve_ground()
        assert abs(e - ref.ecorr) < 1e-9 * abs(ref.ecorr)
        c.solve_lambda()
        c.solve_response(omegas)
        assert _relerr(c.alpha(len(omegas)), ref.alpha) < tol, (prec, ladder)
        c.solve_response(omegas, quadratic=True)
        assert _relerr(c.alpha(len(omegas)), ref.alpha) < tol, (prec, ladder, "eq36")
        c.close()


def test_lean_layout_c3_matches_stored_oracle(monkeypatch):
    """o=20, v=150 with 64 MiB chunks (the FP64 <ov||vv> block is 1.1 GB, so
    every contraction with it runs in 20 chunks): Omega, A X and X A at the
    probe vectors in a 48-vector batch against the stored oracle entries,
    FP64 and mixed (FP32 W resident, FP64 ladder rebuilt from the factors)."""
    from paper_2503_23144_amd.synth import config_inputs, probe_vectors
    monkeypatch.setenv("LRCC_VIRTUAL_CHUNK_BYTES", str(64 << 20))
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "oracle_c3.npz"))
    inp = config_inputs("c3")
    c = _ctx(inp, precision="mixed", tol=1e-11, memory="lean", ladder="full", ladder_fp64="direct")
    t, X, idx = probe_vectors(c.n, int(ref["sig_seed"]))
    R = c.sigma("residual", t)
    assert _relerr(R[idx], ref["sig_residual"]) < 1e-12
    c.set_amplitudes(_lrcc().AMP_T, t)
    rng = np.random.default_rng(99)
    batch = np.concatenate([X[None], _rand(rng, 47, c.n)])
    kl = ref["sig_left_idx"]
    for prec, tol in (("fp64", 1e-12), ("mixed", 2e-6)):
        print(f"lean c3 {prec}", flush=True)
        AX = c.sigma("right", batch, precision=prec)[0]
        assert _relerr(AX[idx], ref["sig_right"]) < tol, prec
        assert abs(np.linalg.norm(AX) / float(ref["sig_right_norm"]) - 1) < tol, prec
        XA = c.sigma("left", batch, precision=prec)[0]
        assert _relerr(XA[kl], ref["sig_left_entries"]) < 10 * tol, prec
    del batch
    e, st = c.solve_ground()
    assert st["converged"] == 1
    assert abs(e - complex(ref["ecorr"])) < 1e-9 * abs(complex(ref["ecorr"]))
