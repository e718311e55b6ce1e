"""Host-side checks of liblrcc.so (no GPU needed).

* the library loads and exports every function include/lrcc.h declares;
* calls fail cleanly (error code + message, no crash) without a device;
* the operation lists the library derives from its CCSD program (right
  sigma, left sigma, xi, dE/dt, grad L and the eta + F X tangent), executed
  op by op with numpy by tests/program_interp.py, equal the oracle's
  autograd/contour-rule derivatives.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle.response import (F_times, Problem, eta, eta0, grad_L, left_sigma, right_sigma, xi)
from paper_2503_23144_amd.synth import make_inputs
from program_interp import Interp, blocks_from_df, fock_blocks, parse


def _lrcc():
    from paper_2503_23144_amd import lrcc
    return lrcc


def test_library_exports_every_declared_symbol():
    lrcc = _lrcc()
    names = lrcc.declared_symbols()
    assert len(names) >= 20
    missing = [s for s in names if not hasattr(lrcc.lib, s)]
    assert not missing, missing
    assert "gfx950" in lrcc.build_info()


def test_default_config():
    lrcc = _lrcc()
    c = lrcc.Config()
    lrcc.lib.lrcc_default_config(ctypes.byref(c))
    assert c.precision == lrcc.FP64 and c.tol_residual == 1e-10 and c.diis_size == 8 and c.maxit == 100
    assert c.autotune == 1


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device error path")
def test_create_without_device_fails_cleanly():
    lrcc = _lrcc()
    h = ctypes.c_void_p()
    rc = lrcc.lib.lrcc_create(ctypes.byref(h), None)
    assert rc in (lrcc.E_HIP, lrcc.E_INVALID)
    assert h.value is None
    assert len(lrcc.lib.lrcc_last_error(None)) > 0
    # calls on a null context are rejected, not crashed
    assert lrcc.lib.lrcc_solve_ground(None, None, None) == lrcc.E_INVALID
    assert lrcc.lib.lrcc_amplitude_length(None) == 0


def test_argument_checks_come_before_any_device_work():
    """Invalid arguments are rejected with LRCC_E_INVALID and a message
    before the library touches a device, so these run on any host."""
    lrcc = _lrcc()
    lib = lrcc.lib
    one = (ctypes.c_double * 2)(1.0, 0.0)
    dummy = ctypes.c_void_p(64)  # never dereferenced: every call below fails its checks first
    cases = [
        (7, 0, 0, 4, 4, 4, 4, 4, 4),     # unknown precision
        (lrcc.FP64, 0, 0, -1, 4, 4, 4, 4, 4),  # negative size
        (lrcc.FP64, 0, 0, 4, 4, 8, 4, 4, 4),   # lda shorter than a row of A (k = 8)
        (lrcc.MIXED, 0, 1, 4, 4, 8, 8, 4, 4),  # ldb shorter than a row of B^T (k = 8)
        (lrcc.MIXED, 0, 0, 4, 8, 4, 4, 8, 4),  # ldc shorter than a row of C (n = 8)
    ]
    for prec, ta, tb, m, n, k, lda, ldb, ldc in cases:
        rc = lib.lrcc_gemm(prec, ta, tb, m, n, k, one, dummy, lda, dummy, ldb, one, dummy, ldc, None)
        assert rc == lrcc.E_INVALID, (prec, m, n, k, lda, ldb, ldc)
        assert len(lib.lrcc_last_error(None)) > 0
    assert lib.lrcc_gemm(lrcc.FP64, 0, 0, 4, 4, 4, one, None, 4, dummy, 4, one, dummy, 4, None) == lrcc.E_INVALID
    assert lib.lrcc_gemm_set_tile(5) == lrcc.E_INVALID and lib.lrcc_gemm_set_tile(-2) == lrcc.E_INVALID
    for field, bad in (("precision", 5), ("ladder_mode", 3), ("tol_residual", 0.0), ("maxit", 0),
                       ("diis_size", 33), ("rhs_chunk", -1), ("ladder_mode_fp64", 3), ("memory_mode", 3),
                       ("ring_factored", 2), ("keep_response", 2)):
        c = lrcc.Config()
        lib.lrcc_default_config(ctypes.byref(c))
        setattr(c, field, bad)
        h = ctypes.c_void_p()
        assert lib.lrcc_create(ctypes.byref(h), ctypes.byref(c)) == lrcc.E_INVALID, field
        assert h.value is None
    assert lib.lrcc_set_workspace(None, dummy, 1 << 30) == lrcc.E_INVALID


def test_program_text_is_well_formed():
    lrcc = _lrcc()
    for which in range(12):
        tensors, ops = parse(lrcc.program_text(which))
        assert ops, which
        for op in ops:
            assert op["out"] in tensors
    assert lrcc.lib.lrcc_program_text(99, None, 0) == -1
    assert lrcc.lib.lrcc_program_text(12, None, 0) == -1


def test_tuned_tile_query_without_a_gpu():
    """lrcc_gemm_tuned_tile is a host lookup: -1 for shapes never timed and
    for invalid arguments."""
    lrcc = _lrcc()
    assert lrcc.gemm_tuned_tile("mixed", 0, 1, 3120, 79800, 79800, ladder=True) == -1
    assert lrcc.lib.lrcc_gemm_tuned_tile(7, 0, 1, 10, 10, 10, 0) == -1
    assert lrcc.lib.lrcc_gemm_tuned_tile(lrcc.FP64, 0, 1, 0, 10, 10, 0) == -1


def _batch(lay, vecs):
    return (np.stack([lay.split(x)[0].numpy() for x in vecs]), np.stack([lay.split(x)[1].numpy() for x in vecs]))


def _cat(env, I, a, b, nb=None):
    if nb is None:
        return np.concatenate([env[I.id(a)].ravel(), env[I.id(b)].ravel()])
    return [np.concatenate([env[I.id(a)][r].ravel(), env[I.id(b)][r].ravel()]) for r in range(nb)]


@pytest.mark.parametrize("o,v,naux,seed", [(3, 5, 8, 4), (2, 7, 6, 9), (4, 4, 5, 1)])
def test_derived_operation_lists_match_oracle(o, v, naux, seed):
    lrcc = _lrcc()
    inp = make_inputs(o, v, naux, seed=seed)
    B = inp.B * 8
    rng = np.random.default_rng(seed)
    fock = inp.fock + 0.05 * (lambda M: M + M.conj().T)(rng.standard_normal((o + v,) * 2) + 0j)
    P = Problem.from_arrays(B, fock, inp.mu, o)
    n = P.lay.n
    nb = 2
    t = torch.as_tensor(0.05 * (rng.standard_normal(n) + 1j * rng.standard_normal(n)))
    tens, res_ops = parse(lrcc.program_text(lrcc.PROG_RESIDUAL))
    I = Interp(tens, o, v, nb)
    env = {}
    for k, val in {**blocks_from_df(B, o), **fock_blocks(fock, o)}.items():
        env[I.id(k)] = val
    t1, t2p = P.lay.split(t)
    env[I.id("t1")], env[I.id("t2p")], env[I.id("one")] = t1.numpy(), t2p.numpy(), np.array(1.0 + 0j)
    I.run(res_ops, env)
    ref = P.omega(t).numpy()
    assert np.abs(_cat(env, I, "O1", "O2p") - ref).max() < 1e-13 * np.abs(ref).max()
    assert abs(complex(env[I.id("E")]) - complex(P.energy(t))) < 1e-14

    X = [torch.as_tensor(rng.standard_normal(n) + 1j * rng.standard_normal(n)) for _ in range(nb)]
    _, right = parse(lrcc.program_text(lrcc.PROG_RIGHT))
    env[I.id("R(t1)")], env[I.id("R(t2p)")] = _batch(P.lay, X)
    I.run(right, env)
    for r, g in enumerate(_cat(env, I, "R(O1)", "R(O2p)", nb)):
        ref = right_sigma(P, t, X[r]).resolve_conj().numpy()
        assert np.abs(g - ref).max() < 1e-12 * np.abs(ref).max()

    _, left = parse(lrcc.program_text(lrcc.PROG_LEFT))
    env[I.id("L(O1)")], env[I.id("L(O2p)")] = _batch(P.lay, X)
    I.run(left, env)
    for r, g in enumerate(_cat(env, I, "L(t1)", "L(t2p)", nb)):
        ref = left_sigma(P, t, X[r]).resolve_conj().numpy()
        assert np.abs(g - ref).max() < 1e-12 * np.abs(ref).max()

    # the factored ring terms: Z1, Z2 formed once from t, then the variants
    _, setup = parse(lrcc.program_text(lrcc.PROG_RING_SETUP))
    I.run(setup, env)
    _, right_f = parse(lrcc.program_text(lrcc.PROG_RIGHT_F))
    env[I.id("R(t1)")], env[I.id("R(t2p)")] = _batch(P.lay, X)
    I.run(right_f, env)
    for r, g in enumerate(_cat(env, I, "R(O1)", "R(O2p)", nb)):
        ref = right_sigma(P, t, X[r]).resolve_conj().numpy()
        assert np.abs(g - ref).max() < 1e-12 * np.abs(ref).max()
    _, left_f = parse(lrcc.program_text(lrcc.PROG_LEFT_F))
    env[I.id("L(O1)")], env[I.id("L(O2p)")] = _batch(P.lay, X)
    I.run(left_f, env)
    for r, g in enumerate(_cat(env, I, "L(t1)", "L(t2p)", nb)):
        ref = left_sigma(P, t, X[r]).resolve_conj().numpy()
        assert np.abs(g - ref).max() < 1e-12 * np.abs(ref).max()
    # neither variant forms the tangent / adjoint of W_mbej (the o^3 v^3 ring
    # contraction with it is what the via terms replace); the plain ones do
    tens_all, _ = parse(lrcc.program_text(lrcc.PROG_LEFT_F))
    nm = lambda k: tens_all[k]["name"] if k >= 0 else ""
    for ops_f, ops_p, wname in ((right_f, right, "R(Wmbej)"), (left_f, left, "L(Wmbej)")):
        assert not any(wname in (nm(op["a"]), nm(op["b"]), nm(op["out"])) for op in ops_f), wname
        assert any(wname in (nm(op["a"]), nm(op["b"]), nm(op["out"])) for op in ops_p), wname

    _, e0 = parse(lrcc.program_text(lrcc.PROG_ETA0))
    I.run(e0, env)
    ref = eta0(P, t).resolve_conj().numpy()
    assert np.abs(_cat(env, I, "E(t1)", "E(t2p)") - ref).max() < 1e-13 * np.abs(ref).max()

    comps = [0, 2]
    _, xip = parse(lrcc.program_text(lrcc.PROG_XI))
    for nm in ("foo", "fov", "fvo", "fvv"):
        env[I.id(f"X({nm})")] = np.stack([fock_blocks(inp.mu[c], o)[nm] for c in comps])
    I.run(xip, env)
    for r, g in enumerate(_cat(env, I, "X(O1)", "X(O2p)", nb)):
        ref = xi(P, t, comps[r]).resolve_conj().numpy()
        assert np.abs(g - ref).max() < 1e-13 * np.abs(ref).max()

    lam = torch.as_tensor(0.02 * (rng.standard_normal(n) + 1j * rng.standard_normal(n)))
    _, gl = parse(lrcc.program_text(lrcc.PROG_GRADL))
    l1, l2 = P.lay.split(lam)
    env[I.id("lam1")], env[I.id("lam2p")] = l1.numpy(), l2.numpy()
    I.run(gl, env)
    ref = grad_L(P, t, lam).resolve_conj().numpy()
    assert np.abs(_cat(env, I, "G(t1)", "G(t2p)") - ref).max() < 1e-13 * np.abs(ref).max()

    _, hv = parse(lrcc.program_text(lrcc.PROG_HVP))
    env[I.id("H(t1)")], env[I.id("H(t2p)")] = _batch(P.lay, X)
    for nm in ("foo", "fov", "fvo", "fvv"):
        env[I.id(f"H({nm})")] = np.stack([fock_blocks(inp.mu[c], o)[nm] for c in comps])
    I.run(hv, env)
    for r, g in enumerate(_cat(env, I, "H(G(t1))", "H(G(t2p))", nb)):
        ref = (F_times(P, t, lam, X[r]) + eta(P, t, lam, comps[r])).resolve_conj().numpy()
        assert np.abs(g - ref).max() < 1e-12 * np.abs(ref).max()

    _, fx = parse(lrcc.program_text(lrcc.PROG_FX))
    env[I.id("F(t1)")], env[I.id("F(t2p)")] = _batch(P.lay, X)
    I.run(fx, env)
    for r, g in enumerate(_cat(env, I, "F(G(t1))", "F(G(t2p))", nb)):
        ref = F_times(P, t, lam, X[r]).resolve_conj().numpy()
        assert np.abs(g - ref).max() < 1e-12 * np.abs(ref).max()


def test_executor_regrouping_leaves_every_program_unchanged():
    """The executor may run a run of permute-accumulates grouped by output
    tensor (its summed permutes); executed in that order with numpy, every
    derived program writes exactly the same tensors as in list order, and the
    regrouping does change the order of some program."""
    import copy

    from program_interp import executor_order
    lrcc = _lrcc()
    o, v, nb = 3, 5, 2
    inp = make_inputs(o, v, 8, seed=4)
    B = inp.B * 8
    rng = np.random.default_rng(4)
    P = Problem.from_arrays(B, inp.fock, inp.mu, o)
    n = P.lay.n
    tens, res_ops = parse(lrcc.program_text(lrcc.PROG_RESIDUAL))
    I = Interp(tens, o, v, nb)
    env = {}
    for k, val in {**blocks_from_df(B, o), **fock_blocks(inp.fock, o)}.items():
        env[I.id(k)] = val
    t = torch.as_tensor(0.05 * (rng.standard_normal(n) + 1j * rng.standard_normal(n)))
    t1, t2p = P.lay.split(t)
    env[I.id("t1")], env[I.id("t2p")], env[I.id("one")] = t1.numpy(), t2p.numpy(), np.array(1.0 + 0j)
    l1, l2 = P.lay.split(torch.as_tensor(0.02 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))))
    env[I.id("lam1")], env[I.id("lam2p")] = l1.numpy(), l2.numpy()
    X = [torch.as_tensor(rng.standard_normal(n) + 1j * rng.standard_normal(n)) for _ in range(nb)]
    for pre in ("R", "L", "H", "F"):
        x1, x2 = _batch(P.lay, X)
        src = ("L(O1)", "L(O2p)") if pre == "L" else (f"{pre}(t1)", f"{pre}(t2p)")
        env[I.id(src[0])], env[I.id(src[1])] = x1, x2
    for nm in ("foo", "fov", "fvo", "fvv"):
        blk = np.stack([fock_blocks(inp.mu[c], o)[nm] for c in (0, 2)])
        env[I.id(f"X({nm})")] = blk
        env[I.id(f"H({nm})")] = blk
    changed = 0
    for which in (lrcc.PROG_RESIDUAL, lrcc.PROG_RIGHT, lrcc.PROG_LEFT, lrcc.PROG_ETA0, lrcc.PROG_XI,
                  lrcc.PROG_GRADL, lrcc.PROG_HVP, lrcc.PROG_FX):
        _, ops = parse(lrcc.program_text(which))
        order = executor_order(ops)
        assert sorted(map(id, order)) == sorted(map(id, ops))
        changed += order != ops
        e1, e2 = I.run(ops, copy.deepcopy(env)), I.run(order, copy.deepcopy(env))
        for k in {op["out"] for op in ops}:
            assert np.array_equal(e1[k], e2[k]), (which, tens[k]["name"])
        env = e1
    assert changed >= 2
    # synthetic runs where the conditions decide (ids: 10, 11, 12 written; 20, 21 read only)
    add = lambda out, a, acc: dict(kind=0, acc=acc, alpha=1.0, out=out, oi="ab", a=a, ai="ab", b=-1, bi="", m=(0, 0))
    zero = lambda out: dict(kind=4, acc=False, alpha=1.0, out=out, oi="ab", a=-1, ai="", b=-1, bi="", m=(0, 0))
    pre = [zero(10), zero(11)]  # 10 and 11 written before the runs
    free = pre + [add(10, 20, True), add(11, 21, True), add(10, 21, True)]
    assert [op["out"] for op in executor_order(free)[2:]] == [10, 10, 11]  # regrouped by output
    reads = pre + [add(10, 20, True), add(11, 10, True), add(10, 21, True)]  # 11 reads 10 mid-run
    assert executor_order(reads) == reads
    first = pre + [add(10, 20, True), add(12, 21, False), add(10, 21, True)]  # 12 first written mid-run
    assert executor_order(first) == first


def test_fnspp_projection_list_matches_oracle():
    """The FNS++ numerators (Eq. 48 and the singles projection), before the
    denominators of Eqs. 46-47 are applied."""
    from oracle.fnspp import mp2_and_hbar, perturbed_amplitudes
    lrcc = _lrcc()
    o, v = 3, 6
    inp = make_inputs(o, v, 8, seed=3)
    B = inp.B * 8
    t2, Hii, Haa = mp2_and_hbar(B, inp.fock, o)
    # with a zero frequency and unit denominators the oracle returns the numerators
    one_i, one_a = torch.zeros_like(Hii), torch.full_like(Haa, 0.5)
    tA1, tA2 = perturbed_amplitudes(t2, one_i, one_a, inp.mu[1], o, 0.0)
    tens, ops = parse(lrcc.program_text(lrcc.PROG_FNSPP))
    I = Interp(tens, o, v, 1)
    blk = fock_blocks(inp.mu[1], o)
    env = {I.id("tm2"): t2.numpy(), I.id("Aoo"): blk["foo"], I.id("Aov"): blk["fov"], I.id("Avo"): blk["fvo"],
           I.id("Avv"): blk["fvv"]}
    I.run(ops, env)
    assert np.abs(env[I.id("s1")] - 0.5 * tA1.numpy()).max() < 1e-14
    assert np.abs(env[I.id("s2")] - tA2.numpy()).max() < 1e-14


def test_workspace_estimate_fits_largest_config_in_lean_layout():
    """The footprint estimate of the o=40, v=400 mixed pipeline with one
    right-hand side per batch in the lean layout (FP32 W as its triangle,
    FP64 ladder rebuilt from the factors) fits one MI355X (288 GB), with
    and without the FP32 Z1 of the factored ring terms (20.5 GB, taken by
    default at this size); the resident layout with both full W does not."""
    from paper_2503_23144_amd import lrcc
    kw = dict(precision="mixed", ladder="triangle", ladder_fp64="direct", memory="lean")
    lean = lrcc.workspace_bytes(40, 400, 800, 1, **kw)
    plain = lrcc.workspace_bytes(40, 400, 800, 1, ring_factored=False, **kw)
    both = lrcc.workspace_bytes(40, 400, 800, 1, ring_factored=True, **kw)
    assert 20e9 < lean - plain < 25e9  # FP32 Z1 only: 1.1 x 40 * 400^3 * 8 bytes
    assert 40e9 < both - lean < 50e9  # forced, the FP64 executor's Z1 as well (twice that)
    resident = lrcc.workspace_bytes(40, 400, 800, 1, precision="mixed", memory="resident")
    assert 0 < plain < 250e9 and lean < 265e9 < 288e9 < resident
    # the plain FP64 solver with the rebuilt ladder fits as well
    assert lrcc.workspace_bytes(40, 400, 800, 1, precision="fp64", ladder="direct", memory="lean") < 250e9


def test_bench_uncoupled_alpha_matches_oracle():
    """The bench's independent-particle alpha (the reference of its
    correlated-part error figures) is the oracle's, at two frequencies."""
    import importlib.util
    import os

    from oracle.response import alpha_uncoupled
    spec = importlib.util.spec_from_file_location("bench", os.path.join(os.path.dirname(__file__), "..", "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    inp = make_inputs(3, 7, 5, seed=2)
    got = bench.alpha_uncoupled_ref(inp.fock, inp.mu, inp.o, [0.0, 0.13])
    for k, w in enumerate((0.0, 0.13)):
        ref = alpha_uncoupled(inp.fock, inp.mu, inp.o, w)
        assert np.abs(got[k] - ref).max() < 1e-14 * np.abs(ref).max()


def test_bench_refuses_more_than_one_gpu_and_reads_traffic_by_tile():
    """bench.py runs on one GPU only: --gpus 2 exits with a message and
    status 2 before touching a device.  The traffic figure is read from the
    committed counter summary only for the tile it was measured on."""
    import importlib.util
    import json
    import os
    import subprocess
    import sys
    root = os.path.join(os.path.dirname(__file__), "..")
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
    spec = importlib.util.spec_from_file_location("bench", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t = bench.measured_traffic("c5", 3)
    assert t is not None and t["tile"] == "128x128x8w" and t["bytes_per_launch"] > 5e11
    assert bench.measured_traffic("c5", 0) is None  # not measured on the 64 x 64 tile
    assert bench.measured_traffic("c1", 3) is None
