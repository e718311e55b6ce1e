"""Benchmark: LR-CCSD Jacobian-product throughput on one MI355X.

Headline (default, workload c5: o=40, v=400, naux=800, the largest
configuration, about 30 % of the 1300-virtual spaces the paper truncates):
a step is one batched right Jacobian product (sigma = A X, Eqs. 29-30) over a
chunk of right-hand sides of the 3 dipole directions x 64 frequencies, in
mixed precision (complex FP32 3M products on MFMA, the FP64 diagonal),
inputs resident in HBM.  `value` is sigma evaluations (one per right-hand
side) per second over the timed steps.  Beside it, in the same record:
  * the plain FP64 solver's product (one right-hand side per product, FP64
    4M on MFMA) at the same size, and the mixed / plain ratio;
  * parity at full size: the mixed product against the FP64 one, and the
    adjoint identity u.(A v) = (u A).v with FP64 products;
  * the ladder kernel's roofline (HIP-event time of its launches);
  * a full T -> Lambda -> X, Y -> alpha solve at o=40, v=400 on a subset of
    the frequencies (mixed precision), and alpha by both routes (Eq. 35 and
    Eq. 36);
  * the full pass at o=20, v=150 (integrals, T, Lambda, 48 X and 48 Y,
    alpha) as a secondary figure;
  * the FP64 oracle on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5|c3]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LR sigma evals/s (3 dirs×nω) + ladder TFLOP/s; FP32-3M vs FP64 at fixed α err"
PEAK = {"fp32": 157.3, "fp64": 78.6}  # dense MFMA TFLOP/s (MI355X)


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name") or line.startswith("Socket(s)") or line.startswith("Thread(s) per core"):
                k, v = line.split(":", 1)
                info[k.strip()] = v.strip()
    except Exception:
        pass
    return info


def gemm_source_hash():
    """First 16 hex digits of the SHA-256 of the GEMM kernel's sources
    (gemm.hip, then outmap.h, the epilogue's address maps)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gemm.hip", "outmap.h"):
        h.update(open(os.path.join(ROOT, "paper_2503_23144_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


TILE_NAMES = {0: "64x64", 1: "128x64", 2: "128x128", 3: "128x128x8w", 4: "128x32"}


def measured_traffic(workload, tile=None):
    """HBM bytes per ladder launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, if it was taken for this workload, for the tile the
    ladder ran with (`tile`, 0..4, as lrcc_gemm_tuned_tile reports it) and the
    GEMM source has not changed since (else None)."""
    import re
    name = {"c3": "ladder_o20_v150_hbm_traffic.md", "c5": "ladder_o40_v400_hbm_traffic.md"}.get(workload)
    path = os.path.join(ROOT, "profiles", name or "-")
    if name is None or not os.path.exists(path):
        return None
    for m in re.finditer(r"traffic_bytes_per_launch=(\d+) tile=(\S+) gemm_src_sha256_16=([0-9a-f]{16})",
                         open(path).read()):
        if gemm_source_hash() != m.group(3) or (tile is not None and TILE_NAMES.get(tile) != m.group(2)):
            continue
        return {"bytes_per_launch": int(m.group(1)), "tile": m.group(2), "source": os.path.relpath(path, ROOT)}
    return None


def alpha_uncoupled_ref(fock, mu, o, omegas):
    """The independent-particle polarizability (no two-electron terms, t = 0):
    sum over single excitations i -> a of mu^A_ia mu^B_ai / (D - w) +
    mu^B_ia mu^A_ai / (D + w), D = F_aa - F_ii, shape [nw, ncomp, ncomp].
    alpha is dominated by it on these inputs, so errors are also quoted
    relative to alpha - alpha_uncoupled (the correlated part)."""
    import numpy as np
    e = np.real(np.diag(np.asarray(fock)))
    mu = np.asarray(mu)
    D = e[o:][None, :] - e[:o][:, None]
    out = np.zeros((len(omegas), mu.shape[0], mu.shape[0]), dtype=np.complex128)
    for k, w in enumerate(omegas):
        for A in range(mu.shape[0]):
            for B in range(mu.shape[0]):
                out[k, A, B] = np.sum(mu[A][:o, o:] * mu[B][o:, :o].T / (D - w)
                                      + mu[B][:o, o:] * mu[A][o:, :o].T / (D + w))
    return out


def correlated_rel_diff(a, ref, unc):
    """max |a - ref| / max |ref - unc|: a difference relative to the part of
    alpha beyond the independent-particle sum."""
    import numpy as np
    return float(np.abs(np.asarray(a) - ref).max() / np.abs(np.asarray(ref) - unc).max())


def resident(inp):
    """The workload's inputs (DF factors, Fock and dipole matrices) as device
    tensors, so that timed passes start from data already in HBM."""
    import torch
    dev = torch.device("cuda:0")
    return {k: torch.as_tensor(getattr(inp, k)).to(dev) for k in ("B", "fock", "mu")}


def run_pass(lrcc, inp, precision, tol, timing=False, chunk=0, dev_in=None, quadratic=False, ladder="full"):
    """One pass of the hot path; returns counts, alpha and phase times.
    dev_in: the inputs already on the device (resident(inp)).  quadratic:
    alpha by the Eq. 36 route (X(w) and X(-w)) instead of Eq. 35 (X and Y)."""
    ph = {}
    src = dev_in if dev_in is not None else {"B": inp.B, "fock": inp.fock, "mu": inp.mu}
    t = time.perf_counter()
    c = lrcc.Context(precision=precision, tol=tol, rhs_chunk=chunk, ladder=ladder)
    c.set_timing(timing)
    c.load_df(inp.o, inp.v, src["B"])
    c.load_fock(src["fock"])
    c.load_dipoles(src["mu"])
    ph["integrals"] = time.perf_counter() - t
    t = time.perf_counter()
    e, st0 = c.solve_ground()
    ph["ground"] = time.perf_counter() - t
    t = time.perf_counter()
    st1 = c.solve_lambda()
    ph["lambda"] = time.perf_counter() - t
    t = time.perf_counter()
    per = c.solve_response(inp.omegas, quadratic=quadratic)
    ph["response"] = time.perf_counter() - t
    resp_sig = sum(s["sigma_evals"] for s in per)
    sig = st0["sigma_evals"] + st1["sigma_evals"] + resp_sig
    alpha = c.alpha(len(inp.omegas))
    ladder = c.kernel_time(0 if precision == "mixed" else 1) if timing else None
    allg = c.kernel_time(2) if timing else None
    c.close()
    return dict(ecorr=e, sigma_evals=sig, resp_sigma_evals=resp_sig, alpha=alpha, ladder=ladder, gemm=allg,
                iters=[s["iterations"] for s in per], phases=ph)


def truncation_curve(lrcc, inp, dev_in, ref_alpha, omega_idx, tol, fracs=(0.25, 0.5, 0.75)):
    """Virtual-space truncation by ground-state natural spinors (FNS, Eq. 40)
    and by perturbation-sensitive ones (FNS++, Eqs. 45-50) at several kept
    fractions: error of the isotropic alpha against the full space, without
    and with the MP2-level correction (Eqs. 53-54), plus the timings.  The
    paper's Fig. 2 comparison, on the synthetic workload."""
    import numpy as np
    omegas = [float(inp.omegas[k]) for k in omega_idx]
    ref = np.asarray(ref_alpha)[list(omega_idx)]
    iso = lambda a: np.real(np.trace(a, axis1=-2, axis2=-1)) / 3.0

    def ctx():
        c = lrcc.Context(precision="mixed", tol=tol)
        c.load_df(inp.o, inp.v, dev_in["B"])
        c.load_fock(dev_in["fock"])
        c.load_dipoles(dev_in["mu"])
        return c

    c = ctx()
    t = time.perf_counter()
    e_full, a_full = c.mp2_response(omegas)
    t_mp2 = time.perf_counter() - t
    c.close()
    rows = []
    for frac in fracs:
        keep = max(2, int(round(frac * inp.v)))
        for scheme in ("fns", "fnspp"):
            c = ctx()
            t = time.perf_counter()
            if scheme == "fns":
                c.fns_truncate(keep=keep)
            else:
                c.fnspp_truncate(omegas, keep=keep)
            t_trunc = time.perf_counter() - t
            e_tr, a_tr = c.mp2_response(omegas)
            t = time.perf_counter()
            e_cc, _ = c.solve_ground()
            c.solve_lambda()
            c.solve_response(omegas)
            t_solve = time.perf_counter() - t
            al = c.alpha(len(omegas))
            c.close()
            rows.append({"scheme": scheme, "kept_virtuals": keep, "kept_fraction": keep / inp.v,
                         "alpha_iso_rel_err": [float(x) for x in np.abs(iso(al) - iso(ref)) / np.abs(iso(ref))],
                         "alpha_iso_rel_err_mp2_corrected": [
                             float(x) for x in np.abs(iso(al + a_full - a_tr) - iso(ref)) / np.abs(iso(ref))],
                         "delta_e_mp2": float(np.real(e_full - e_tr)),
                         "truncate_s": t_trunc, "solve_s": t_solve})
            print(f"[bench] truncation {scheme} keep {keep}: alpha_iso err {rows[-1]['alpha_iso_rel_err']}",
                  file=sys.stderr, flush=True)
    return {"omegas": omegas, "mp2_full_space_s": t_mp2, "rows": rows}


def _sampled_entries(A, W, C, dt, count=48):
    """Parity of C = A W^T at full size on sampled entries: each entry is
    recomputed on the host as a complex128 dot product of one row of A and
    one row of W, and its error is compared with the dot-product rounding
    scale eps * sum_k |A_ik| |W_jk| (eps of the GEMM's precision)."""
    import numpy as np
    import torch
    g = np.random.default_rng(17)
    ii = g.integers(0, A.shape[0], count)
    jj = g.integers(0, W.shape[0], count)
    ar = A[torch.as_tensor(ii, device=A.device)].cpu().numpy().astype(np.complex128)
    wr = W[torch.as_tensor(jj, device=W.device)].cpu().numpy().astype(np.complex128)
    got = C[torch.as_tensor(ii, device=C.device), torch.as_tensor(jj, device=C.device)].cpu().numpy()
    ref = np.einsum("sk,sk->s", ar, wr)
    scale = np.einsum("sk,sk->s", np.abs(ar), np.abs(wr))
    eps = 2.0 ** -24 if dt == torch.complex64 else 2.0 ** -53
    ratio = float(np.max(np.abs(got - ref) / (eps * scale)))
    # rounding grows like sqrt(K) for random data; 4 sqrt(K) is far below the
    # worst-case K and far above what a wrong index or a dropped term gives
    bound = 4.0 * np.sqrt(A.shape[1])
    ok = ratio <= bound
    print(f"[bench]   sampled entries: max |err| / (eps sum|a||b|) = {ratio:.2f} (bound {bound:.0f})",
          file=sys.stderr, flush=True)
    assert ok, "ladder GEMM at scale disagrees with the host dot products"
    return {"entries": count, "max_err_over_eps_scale": ratio, "bound": bound, "ok": bool(ok)}


def gemm_probe(lrcc, o=20, v=150, nrhs=48, tile=0, calibrate=False):
    """C = A W^T with the shape of a batched ladder (M = nrhs * o(o-1)/2,
    N = K = v(v-1)/2, complex64), three launches with one pinned workgroup
    tile; prints each launch time.  calibrate: first one plain 1 GiB device
    copy, the reference for the HBM byte counters."""
    import torch
    dev = torch.device("cuda:0")
    if calibrate:
        src = torch.ones(2**27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 1 GiB read, 1 GiB written", file=sys.stderr, flush=True)
        del src, dst
    if nrhs == 0:
        return
    po, pv = o * (o - 1) // 2, v * (v - 1) // 2
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    A = torch.randn(nrhs * po, pv, dtype=torch.complex64, device=dev, generator=g)
    W = torch.randn(pv, pv, dtype=torch.complex64, device=dev, generator=g)
    C = torch.empty(nrhs * po, pv, dtype=torch.complex64, device=dev)
    lrcc.gemm_set_tile(tile)
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        lrcc.gemm(A, W, C, transb=True)
        e1.record()
        torch.cuda.synchronize()
        print(f"[bench] gemm probe {A.shape[0]} x {pv} x {pv} tile {tile}: {e0.elapsed_time(e1):.2f} ms",
              file=sys.stderr, flush=True)
    lrcc.gemm_set_tile(-1)


def ladder_at_scale(lrcc, o=40, v=400, nrhs=4, reps=3):
    """The particle-particle ladder sum_{e<f} <ab||ef> tau_ij^ef of one batched
    sigma at o=40, v=400: C[(r,i<j)][a<b] = taup[(r,i<j)][e<f] W[a<b][e<f]
    with the packed vvvv matrix W (79800 x 79800) resident in HBM, as complex
    FP32 (3M) and complex FP64 (4M).  Operand values do not change the work;
    they are seeded random numbers here."""
    import torch
    dev = torch.device("cuda:0")
    lrcc.trim_memory()  # the library's cached blocks back to the device before torch allocates W
    po, pv = o * (o - 1) // 2, v * (v - 1) // 2
    M, N, K = nrhs * po, pv, pv
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    out = {"o": o, "v": v, "rhs": nrhs, "m": M, "n": N, "k": K}
    for name, dt, mult, peak in (("fp32_3m", torch.complex64, 6, PEAK["fp32"]),
                                 ("fp64_4m", torch.complex128, 8, PEAK["fp64"])):
        W = torch.randn(N, K, dtype=dt, device=dev, generator=g)
        A = torch.randn(M, K, dtype=dt, device=dev, generator=g)
        C = torch.empty(M, N, dtype=dt, device=dev)
        lrcc.gemm(A, W, C, transb=True)  # warm-up (and tile autotuning)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lrcc.gemm(A, W, C, transb=True)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        t = sorted(ts)[len(ts) // 2]
        tf = mult * M * N * K / t / 1e12
        out[name] = {"ms": 1e3 * t, "tflops": tf, "peak": peak, "frac": tf / peak,
                     "w_gib": W.numel() * W.element_size() / 2**30,
                     "sampled_check": _sampled_entries(A, W, C, dt)}
        print(f"[bench] ladder o={o} v={v} {name}: {1e3 * t:.1f} ms, {tf:.1f} TFLOP/s ({100 * tf / peak:.1f}% of peak)",
              file=sys.stderr, flush=True)
        del W, A, C
        torch.cuda.empty_cache()
    out["fp32_3m_over_fp64_4m_time"] = out["fp64_4m"]["ms"] / out["fp32_3m"]["ms"]
    return out


def _product_rates(lrcc, inp, nvec, graphs, stream, min_s=0.5):
    """Right products per second on one context: (label -> rate)."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    rates = {}
    with torch.cuda.stream(stream):
        c = lrcc.Context(precision="mixed", graphs=graphs, stream=stream.cuda_stream)
        c.load_df(inp.o, inp.v, inp.B)
        c.load_fock(inp.fock)
        c.load_dipoles(inp.mu)
        n = c.n
        rng = np.random.default_rng(5)
        c.set_amplitudes(lrcc.AMP_T, 0.05 * (rng.standard_normal(n) + 1j * rng.standard_normal(n)))
        X = torch.tensor(rng.standard_normal((nvec, n)) + 1j * rng.standard_normal((nvec, n)),
                         dtype=torch.complex128, device=dev)
        out = torch.empty_like(X)
        cases = [("fp64_plain", 1, "fp64")]
        if graphs:
            cases += [("fp64_batched", nvec, "fp64"), ("mixed_batched", nvec, "mixed")]
        for label, nb, prec in cases:
            for w in range(2):  # eager run (and tile tuning), then graph capture
                tw = time.perf_counter()
                c.sigma("right", X[:nb], precision=prec, out=out[:nb])
                stream.synchronize()
                print(f"[bench]   o={inp.o} v={inp.v} {label} warm-up {w}: {time.perf_counter() - tw:.1f} s",
                      file=sys.stderr, flush=True)
            k, t0 = 0, time.perf_counter()
            while k < 3 or time.perf_counter() - t0 < min_s:
                c.sigma("right", X[:nb], precision=prec, out=out[:nb])
                k += 1
                if k % 8 == 0 or nb > 1:
                    stream.synchronize()
            stream.synchronize()
            rates[label] = k * nb / (time.perf_counter() - t0)
            print(f"[bench]   o={inp.o} v={inp.v} {label}{'' if graphs else ' (no graphs)'}: {rates[label]:.4g} /s",
                  file=sys.stderr, flush=True)
        if graphs:
            # parity at this size by properties that hold at any size, in the
            # batched launch configuration timed above: the adjoint identity
            # u.(A v) = (u A).v in FP64, and the mixed product against FP64
            c.sigma("right", X, precision="fp64", out=out)
            r64 = out[:2].clone()
            c.sigma("right", X, precision="mixed", out=out)
            r32 = out[:2].clone()
            lt = torch.empty_like(X[:1])
            c.sigma("left", X[1:2], precision="fp64", out=lt)
            stream.synchronize()
            lhs, rhs = complex((X[1] * r64[0]).sum()), complex((lt[0] * X[0]).sum())
            rates["check_adjoint_identity_rel"] = abs(lhs - rhs) / abs(lhs)
            rates["check_mixed_vs_fp64_rel"] = float((r32 - r64).abs().max() / r64.abs().max())
            print(f"[bench]   o={inp.o} v={inp.v} checks: adjoint identity {rates['check_adjoint_identity_rel']:.1e}, "
                  f"mixed vs FP64 {rates['check_mixed_vs_fp64_rel']:.1e}", file=sys.stderr, flush=True)
            assert rates["check_adjoint_identity_rel"] < 1e-10 and rates["check_mixed_vs_fp64_rel"] < 2e-5, \
                "Jacobian products at this size fail their property checks"
            del r64, r32, lt
        c.close()
    del X, out
    lrcc.trim_memory()
    torch.cuda.empty_cache()
    return rates


def sigma_rates(lrcc, names=("c1", "c2", "c3", "c4"), max_batch={"c4": 16}):
    """Jacobian products (A X) per second at each workload shape: FP64 one
    right-hand side per product (the plain solver's product), FP64 batched,
    and mixed-precision batched (FP32 3M coupling products + FP64 diagonal);
    the batch is 3 dipole directions x n_w frequencies (capped at 48, and at
    16 for o=30, v=300, per product).  Amplitudes T and X are seeded random
    vectors resident on the device.  The plain product is also timed with
    HIP graph replay off."""
    import torch

    from paper_2503_23144_amd.synth import CONFIGS, config_inputs
    lrcc.trim_memory()
    stream = torch.cuda.Stream()  # graphs are captured on the caller's stream unless it is the null stream
    table = {}
    for name in names:
        cfg = CONFIGS[name]
        inp = config_inputs(name)
        nvec = min(3 * len(cfg["omegas"]), max_batch.get(name, 48))
        row = {"o": inp.o, "v": inp.v, "batch": nvec}
        row.update(_product_rates(lrcc, inp, nvec, True, stream))
        row["fp64_plain_no_graphs"] = _product_rates(lrcc, inp, nvec, False, stream)["fp64_plain"]
        row["mixed_batched_over_fp64_plain"] = row["mixed_batched"] / row["fp64_plain"]
        row["graph_speedup_fp64_plain"] = row["fp64_plain"] / row["fp64_plain_no_graphs"]
        print(f"[bench] sigma rates {name}: " + ", ".join(f"{k}={v:.3g}" for k, v in row.items()
                                                          if isinstance(v, float)), file=sys.stderr, flush=True)
        table[name] = row
    return table


def cpu_baseline(inp, budget_s=25.0):
    """The oracle, as it stands, timed on the host: right-sigma (A X)
    evaluations at the workload's shapes, one right-hand side at a time."""
    import numpy as np
    import torch

    from oracle.response import Problem, right_sigma, solve_ground
    P = Problem.from_arrays(inp.B, inp.fock, inp.mu, inp.o)
    rng = np.random.default_rng(7)
    n = P.lay.n
    t = torch.as_tensor(0.01 * (rng.standard_normal(n) + 1j * rng.standard_normal(n)))
    X = torch.as_tensor(rng.standard_normal(n) + 1j * rng.standard_normal(n))
    print("[bench] cpu baseline: oracle integral build (not timed)", file=sys.stderr, flush=True)
    P.g("vvvv")  # integral build is not timed
    right_sigma(P, t, X)  # warm
    print("[bench] cpu baseline: timing oracle right sigmas", file=sys.stderr, flush=True)
    k, t0 = 0, time.perf_counter()
    while True:
        right_sigma(P, t, X)
        k += 1
        if time.perf_counter() - t0 > budget_s or k >= 50:
            break
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "sigma evals/s", "cores": torch.get_num_threads(), "kind": "oracle",
            "sample": f"{k} right-sigma (A X) evaluations of the FP64 oracle at o={inp.o}, v={inp.v}, one RHS each, "
                      f"integral build excluded ({dt:.1f} s)"}


def _c5_context(lrcc, inp, dev_in, precision, ladder, ladder_fp64=None, tol=1e-6, chunk=0, ring=None, keep=True,
                verbose=None):
    if verbose is None:  # long solves print their progress
        verbose = 1 if not keep else 0
    c = lrcc.Context(precision=precision, tol=tol, ladder=ladder, ladder_fp64=ladder_fp64, memory="lean",
                     rhs_chunk=chunk, ring_factored=ring, keep_response=keep, verbose=verbose)
    c.load_df(inp.o, inp.v, dev_in["B"])
    c.load_fock(dev_in["fock"])
    c.load_dipoles(dev_in["mu"])
    return c


def _probe_set(n, nb, seed=5):
    """Seeded amplitudes T (0.01 N(0,1) complex) and nb right-hand sides X
    (N(0,1) complex) for the product legs; the work of a Jacobian product
    does not depend on the values."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t = 0.01 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    X = rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))
    return t, X


def sigma_leg(lrcc, inp, dev_in, nb, steps, warmup):
    """The headline: batched mixed-precision right products at full size.
    FP32 W resident (the ladder's operand), the FP64 ladder rebuilt from the
    factors (it serves only FP64 products, none timed here)."""
    import torch
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    c = _c5_context(lrcc, inp, dev_in, "mixed", "full", "direct")
    t, Xh = _probe_set(c.n, nb)
    c.set_amplitudes(lrcc.AMP_T, t)
    X = torch.tensor(Xh, dtype=torch.complex128, device=dev)
    out = torch.empty_like(X)
    setup = time.perf_counter() - t0
    print(f"[bench] c5 mixed context ready ({setup:.1f} s), n = {c.n}, batch {nb}", file=sys.stderr, flush=True)
    for w in range(warmup):
        tw = time.perf_counter()
        c.sigma("right", X, precision="mixed", out=out)
        torch.cuda.synchronize()
        print(f"[bench] c5 warmup {w}: {time.perf_counter() - tw:.2f} s", file=sys.stderr, flush=True)
    c.set_timing(True)  # HIP events around every GEMM launch, on the executor's stream
    torch.cuda.synchronize()
    ts = time.perf_counter()
    ladder, allg = [0.0, 0, 0.0], [0.0, 0, 0.0]
    for k in range(steps):
        c.sigma("right", X, precision="mixed", out=out)
        torch.cuda.synchronize()
        for acc, cls in ((ladder, 0), (allg, 2)):  # each product reports its own launches
            for q, x in enumerate(c.kernel_time(cls)):
                acc[q] += x
        print(f"[bench] c5 step {k}: {time.perf_counter() - ts:.2f} s", file=sys.stderr, flush=True)
    dt = time.perf_counter() - ts
    c.set_timing(False)
    row0 = out[0].cpu().numpy()
    c.close()
    del X, out
    lrcc.trim_memory()
    torch.cuda.empty_cache()
    return {"value": steps * nb / dt, "seconds": dt, "steps": steps, "batch": nb, "setup_s": setup,
            "ladder": ladder, "gemm": allg, "row0_mixed": row0, "t": t, "X0": Xh[0], "n": len(t)}


def fp64_plain_leg(lrcc, inp, dev_in, t, X0, reps=3):
    """The plain FP64 solver's product at full size: one right-hand side per
    product, FP64 W resident, the ring's dt1 terms factored as in the mixed
    leg (FP64 Z1, 41 GB; the solver's automatic choice at this size would
    contract them directly).  Also the parity checks at this size: the
    adjoint identity u.(A v) = (u A).v and the FP64 product of the first
    right-hand side for the mixed leg's comparison."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    c = _c5_context(lrcc, inp, dev_in, "fp64", "full", ring=True)
    c.set_amplitudes(lrcc.AMP_T, t)
    X = torch.tensor(X0[None], dtype=torch.complex128, device=dev)
    out = torch.empty_like(X)
    setup = time.perf_counter() - t0
    c.sigma("right", X, precision="fp64", out=out)  # warm-up: tiles of the FP64 shapes
    torch.cuda.synchronize()
    print(f"[bench] c5 fp64 context ready ({setup:.1f} s) and warm", file=sys.stderr, flush=True)
    c.set_timing(True)
    ts = time.perf_counter()
    ladder = [0.0, 0, 0.0]
    for k in range(reps):
        c.sigma("right", X, precision="fp64", out=out)
        torch.cuda.synchronize()
        for q, x in enumerate(c.kernel_time(1)):
            ladder[q] += x
    dt = time.perf_counter() - ts
    c.set_timing(False)
    r64 = out[0].cpu().numpy()
    rng = np.random.default_rng(23)
    U = torch.tensor((rng.standard_normal(c.n) + 1j * rng.standard_normal(c.n))[None], dtype=torch.complex128,
                     device=dev)
    UA = torch.empty_like(U)
    c.sigma("left", U, precision="fp64", out=UA)
    torch.cuda.synchronize()
    lhs = complex((U[0] * out[0]).sum())
    rhs = complex((UA[0] * X[0]).sum())
    c.close()
    del X, out, U, UA
    lrcc.trim_memory()
    torch.cuda.empty_cache()
    print(f"[bench] c5 fp64 plain: {reps / dt:.3f} products/s", file=sys.stderr, flush=True)
    return {"sigma_evals_per_s": reps / dt, "seconds": dt, "products": reps, "setup_s": setup,
            "ladder_tflops": ladder[2] / max(ladder[0] / 1e3, 1e-30) / 1e12, "ladder_ms_per_launch":
            ladder[0] / max(ladder[1], 1), "adjoint_identity_rel": abs(lhs - rhs) / abs(lhs), "row0_fp64": r64}


def solve_leg(lrcc, inp, dev_in, omegas, tol=1e-6, keep_response=True, eq36=True):
    """A full T -> Lambda -> X, Y -> alpha solve at full size in mixed
    precision on a subset of the frequencies (one right-hand side per
    product: the FP32 W as its Hermitian triangle, the FP64 ladder rebuilt,
    so that the solver's buffers fit beside it), then alpha by Eq. 36."""
    import numpy as np
    import torch
    out = {"omegas": list(omegas), "tol_residual": tol, "ladder": "FP32 triangle, FP64 rebuilt from the factors",
           "rhs_per_product": 1}
    t0 = time.perf_counter()
    c = _c5_context(lrcc, inp, dev_in, "mixed", "triangle", "direct", tol=tol, chunk=1, keep=keep_response)
    out["keep_response"] = keep_response
    out["integrals_s"] = time.perf_counter() - t0
    t = time.perf_counter()
    e, st0 = c.solve_ground()
    out["ground"] = {"seconds": time.perf_counter() - t, "ecorr": [e.real, e.imag], "iterations": st0["iterations"]}
    print(f"[bench] c5 solve: ground {out['ground']}", file=sys.stderr, flush=True)
    t = time.perf_counter()
    st1 = c.solve_lambda()
    out["lambda"] = {"seconds": time.perf_counter() - t, "iterations": st1["iterations"]}
    t = time.perf_counter()
    per = c.solve_response(omegas)
    out["response"] = {"seconds": time.perf_counter() - t, "iterations": [p["iterations"] for p in per],
                       "sigma_evals": int(sum(p["sigma_evals"] for p in per)),
                       "converged": bool(all(p["converged"] for p in per))}
    a35 = c.alpha(len(omegas))
    print(f"[bench] c5 solve: response {out['response']}", file=sys.stderr, flush=True)
    a36 = None
    if eq36:
        t = time.perf_counter()
        per = c.solve_response(omegas, quadratic=True)
        out["eq36"] = {"seconds": time.perf_counter() - t, "converged": bool(all(p["converged"] for p in per))}
        a36 = c.alpha(len(omegas))
    c.close()
    lrcc.trim_memory()
    torch.cuda.empty_cache()
    out["alpha_iso"] = [float(x) for x in np.real(np.trace(a35, axis1=-2, axis2=-1)) / 3.0]
    out["alpha"] = [[[complex(z).real, complex(z).imag] for z in row] for row in np.asarray(a35[0])]
    if len(omegas) > 1:
        out["alpha_all"] = [[[[complex(z).real, complex(z).imag] for z in row] for row in ak] for ak in np.asarray(a35)]
    out["alpha_max_asymmetry_static"] = (float(np.abs(a35[0] - a35[0].T).max() / np.abs(a35[0]).max())
                                         if omegas[0] == 0.0 else None)
    if a36 is not None:
        out["alpha_rel_diff_eq36_vs_eq35"] = float(np.abs(a36 - a35).max() / np.abs(a35).max())
        out["alpha_rel_diff_eq36_vs_eq35_correlated_part"] = correlated_rel_diff(
            a36, a35, alpha_uncoupled_ref(inp.fock, inp.mu, inp.o, omegas))
    out["seconds"] = time.perf_counter() - t0
    print(f"[bench] c5 solve: {out['seconds']:.1f} s, eq36 vs eq35 {out.get('alpha_rel_diff_eq36_vs_eq35')}",
          file=sys.stderr, flush=True)
    return out, a35


def cpu_baseline_scaled(budget_s=25.0):
    """The oracle, as it stands, on the host cores.  It holds dense vvvv
    (410 GB at o=40, v=400), so it is timed at o=20, v=150 (one right-hand
    side per product) and its rate scaled to o=40, v=400 by the ratio of the
    estimated complex multiply-adds per product."""
    from paper_2503_23144_amd.synth import config_inputs
    inp = config_inputs("c3")
    r = cpu_baseline(inp, budget_s=budget_s)
    macs = lambda o, v: (o * (o - 1) / 2) * (v * (v - 1) / 2) ** 2 + (o * v) ** 3 \
        + o * v * (o * (o - 1) / 2) * (v * (v - 1) / 2) + 2 * (o * (o - 1) / 2) ** 2 * (v * (v - 1) / 2) \
        + 3 * (o ** 2 * v ** 3 + o ** 3 * v ** 2)
    scale = macs(20, 150) / macs(40, 400)
    r["measured_at_o20_v150"] = r["value"]
    r["value"] = r["value"] * scale
    r["sample"] = (r["sample"] + f"; scaled to o=40, v=400 by the estimated complex MACs per product "
                   f"(x{scale:.3g}), i.e. extrapolated")
    r["extrapolated"] = True
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c5", choices=["c5", "c3"])
    ap.add_argument("--chunk", type=int, default=4, help="right-hand sides per batched product (c5)")
    ap.add_argument("--solve-omega", type=float, default=0.25,
                    help="frequency of the full o=40, v=400 solve (3 dipole directions)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 product leg (c5)")
    ap.add_argument("--no-solve", action="store_true", help="skip the full o=40, v=400 solve (c5)")
    ap.add_argument("--no-c3", action="store_true", help="skip the o=20, v=150 full pass (c5)")
    ap.add_argument("--c4-check", action="store_true",
                    help="only the o=30, v=300 check: mixed solves of all 3 x 32 right-hand sides by Eq. 35 and "
                         "Eq. 36, and plain FP64 solves on 4 of the 32 frequencies for comparison")
    ap.add_argument("--solve-omegas", type=int, default=1,
                    help="c5 solve on this many frequencies of the grid (more than 1: alpha per frequency, "
                         "only the last frequency's X and Y kept)")
    ap.add_argument("--solve-range", default="",
                    help="c5 solve on the frequencies lo:hi of the 64-point grid (alpha per frequency)")
    ap.add_argument("--fnspp-scale", action="store_true",
                    help="FNS++ from 1300 virtuals to 400 at o=40, then the static solve in the kept space")
    ap.add_argument("--solve-fp64", action="store_true",
                    help="also the plain FP64 solve at o=40, v=400 on the same frequency, for the mixed-vs-FP64 "
                         "alpha comparison (about 5 minutes)")
    ap.add_argument("--fp64", default="both", choices=["none", "plain", "batched", "both"],
                    help="FP64 comparison passes of the c3 pass: plain (one RHS per product) and/or batched")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--extras", action="store_true",
                    help="also the o=20, v=150 legs: Eq. 36 pass, ladder storage modes, truncation curve, "
                         "per-size product rates, the o=40, v=400 ladder on random operands")
    ap.add_argument("--no-ladder-scale", action="store_true", help="skip the o=40, v=400 ladder measurement")
    ap.add_argument("--no-sigma-table", action="store_true", help="skip the per-workload product rates")
    ap.add_argument("--no-eq36", action="store_true", help="skip the Eq. 36 (X(w), X(-w)) pass")
    ap.add_argument("--no-truncation", action="store_true", help="skip the FNS / FNS++ truncation curve")
    ap.add_argument("--no-ladder-modes", action="store_true",
                    help="skip the passes with the DF-direct and the triangle-stored ladder")
    ap.add_argument("--gemm-probe", action="store_true",
                    help="only launch the ladder GEMM of the workload (c5: 4 x 780 rows of packed doubles "
                         "against the 79800 x 79800 W, FP32 3M) three times, for hardware counter runs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device copy (reference for HBM byte counters)")
    # residual tolerances that meet each path's alpha target (mixed: 1e-6
    # relative on alpha; FP64: 1e-10 on residuals, 1e-8 on alpha)
    ap.add_argument("--tol", type=float, default=1e-6, help="mixed-precision residual tolerance")
    ap.add_argument("--tol64", type=float, default=1e-10, help="FP64 residual tolerance")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if not args.extras:
        args.no_eq36 = args.no_ladder_modes = args.no_truncation = args.no_sigma_table = True
        args.no_ladder_scale = True
    if args.c4_check:
        return c4_check(args)
    if args.fnspp_scale:
        return fnspp_scale(args)
    if args.workload == "c3":
        return main_full_pass(args)
    main_c5(args)


def fnspp_scale(args):
    """FNS++ at the spectrum scale: o=40 with 1300 virtual spinors generated
    (naux=800, the full space the o=40, v=400 workload stands for), the
    static FNS++ density (Eqs. 45-50; three directions, omega = 0), its
    1300 x 1300 eigensolve, and the 400 natural spinors of largest |n| kept
    (random factors have no physical occupation decay, so a keep-count
    replaces the 1e-5 threshold); then T, Lambda, X and Y (omega = 0, three
    directions) and alpha in the truncated space, mixed precision.  Checks
    that hold at any size: the kept count, the occupations ordered by |n|,
    converged solves, and alpha(0) symmetric."""
    import numpy as np
    import torch

    from paper_2503_23144_amd import lrcc
    from paper_2503_23144_amd.synth import make_inputs_on_device
    o, v, naux, keep = 40, 1300, 800, 400
    out = {"workload": f"fnspp at scale: o={o}, {v} virtuals generated, naux={naux}, keep {keep}; omega = 0",
           "inputs": "B drawn on the device (torch Philox, seed 0); eps, F, mu numpy PCG64 (seed 0)"}
    t0 = time.perf_counter()
    inp = make_inputs_on_device(o, v, naux, seed=0)
    dev_in = {"B": inp.B, "fock": torch.as_tensor(inp.fock).cuda(), "mu": torch.as_tensor(inp.mu).cuda()}
    torch.cuda.synchronize()
    out["inputs_s"] = time.perf_counter() - t0
    print(f"[bench] fnspp scale: inputs drawn ({out['inputs_s']:.1f} s)", file=sys.stderr, flush=True)
    c = lrcc.Context(precision="mixed", tol=args.tol, ladder="triangle", ladder_fp64="direct", memory="lean",
                     rhs_chunk=1)
    c.load_df(o, v, dev_in["B"])
    c.load_fock(dev_in["fock"])
    c.load_dipoles(dev_in["mu"])
    del dev_in, inp
    torch.cuda.empty_cache()
    t = time.perf_counter()
    nk, occ = c.fnspp_truncate([0.0], keep=keep)
    out["truncate_s"] = time.perf_counter() - t
    a = np.abs(occ)
    out["kept"] = int(nk)
    out["occupations"] = {"n_1": float(occ[0]), "n_keep": float(occ[keep - 1]), "n_keep+1": float(occ[keep]),
                          "n_last": float(occ[-1]), "captured_abs_fraction": float(a[:keep].sum() / a.sum()),
                          "negative": int((occ < 0).sum())}
    out["ordered_by_abs"] = bool(np.all(a[:-1] >= a[1:]))
    print(f"[bench] fnspp scale: truncate {out['truncate_s']:.1f} s, kept {nk}, {out['occupations']}",
          file=sys.stderr, flush=True)
    t = time.perf_counter()
    e, st0 = c.solve_ground()
    out["ground"] = {"seconds": time.perf_counter() - t, "ecorr": [e.real, e.imag], "iterations": st0["iterations"],
                     "converged": bool(st0["converged"])}
    print(f"[bench] fnspp scale: ground {out['ground']}", file=sys.stderr, flush=True)
    t = time.perf_counter()
    st1 = c.solve_lambda()
    out["lambda"] = {"seconds": time.perf_counter() - t, "iterations": st1["iterations"],
                     "converged": bool(st1["converged"])}
    print(f"[bench] fnspp scale: lambda {out['lambda']}", file=sys.stderr, flush=True)
    t = time.perf_counter()
    per = c.solve_response([0.0])
    out["response"] = {"seconds": time.perf_counter() - t, "iterations": [p["iterations"] for p in per],
                       "converged": bool(all(p["converged"] for p in per))}
    al = np.asarray(c.alpha(1))[0]
    c.close()
    lrcc.trim_memory()
    out["alpha"] = [[[complex(z).real, complex(z).imag] for z in row] for row in al]
    out["alpha_asymmetry"] = float(np.abs(al - al.T).max() / np.abs(al).max())
    out["seconds"] = time.perf_counter() - t0
    print(f"[bench] fnspp scale: {out['seconds']:.1f} s, alpha asymmetry {out['alpha_asymmetry']:.1e}",
          file=sys.stderr, flush=True)
    print(json.dumps(out))


def c4_check(args):
    """o=30, v=300, naux=600, 3 directions x 32 frequencies in [0, 0.4] Ha:
    the batched mixed solver on every right-hand side (uneven convergence:
    the frequencies approach the first excitation), alpha by Eq. 35 and by
    Eq. 36, and the plain FP64 solver on four of the frequencies."""
    import numpy as np
    import torch

    from paper_2503_23144_amd import lrcc
    from paper_2503_23144_amd.synth import config_inputs
    inp = config_inputs("c4")
    dev_in = resident(inp)
    om = [float(w) for w in inp.omegas]
    out = {"workload": "c4: o=30 v=300 naux=600, 3 dipole directions x 32 omegas in [0,0.4] Ha",
           "gap": inp.gap}

    def ctx(prec, tol):
        c = lrcc.Context(precision=prec, tol=tol, verbose=1)
        c.load_df(inp.o, inp.v, dev_in["B"])
        c.load_fock(dev_in["fock"])
        c.load_dipoles(dev_in["mu"])
        return c

    t0 = time.perf_counter()
    c = ctx("mixed", args.tol)
    c.solve_ground()
    c.solve_lambda()
    out["mixed_ground_lambda_s"] = time.perf_counter() - t0
    t = time.perf_counter()
    per = c.solve_response(om)
    out["mixed_eq35_s"] = time.perf_counter() - t
    a35 = c.alpha(len(om))
    its = [p["iterations"] for p in per]
    out["iterations_x"] = its[:96]
    out["iterations_y"] = its[96:]
    out["sigma_evals_eq35"] = int(sum(p["sigma_evals"] for p in per))
    captures, replays = c.graph_stats()
    out["graph_captures"], out["graph_replays"] = captures, replays
    print(f"[bench] c4 mixed eq35: {out['mixed_eq35_s']:.1f} s, X iterations {min(its[:96])}..{max(its[:96])}",
          file=sys.stderr, flush=True)
    t = time.perf_counter()
    c.solve_response(om, quadratic=True)
    out["mixed_eq36_s"] = time.perf_counter() - t
    a36 = c.alpha(len(om))
    out["alpha_rel_diff_eq36_vs_eq35"] = float(np.abs(a36 - a35).max() / np.abs(a35).max())
    c.close()
    lrcc.trim_memory()
    sub = [0, 10, 21, 31]
    t = time.perf_counter()
    c = ctx("fp64", args.tol64)
    c.solve_ground()
    c.solve_lambda()
    c.solve_response([om[k] for k in sub])
    a64 = c.alpha(len(sub))
    c.close()
    lrcc.trim_memory()
    out["fp64_subset_omegas"] = [om[k] for k in sub]
    out["fp64_s"] = time.perf_counter() - t
    out["alpha_rel_diff_mixed_vs_fp64"] = float(np.abs(a35[sub] - a64).max() / np.abs(a64).max())
    out["alpha_rel_diff_mixed_vs_fp64_correlated_part"] = correlated_rel_diff(
        a35[sub], a64, alpha_uncoupled_ref(inp.fock, inp.mu, inp.o, [om[k] for k in sub]))
    out["alpha_rel_diff_eq36_vs_eq35_correlated_part"] = correlated_rel_diff(
        a36, a35, alpha_uncoupled_ref(inp.fock, inp.mu, inp.o, om))
    out["alpha_iso"] = [float(x) for x in np.real(np.trace(a35, axis1=-2, axis2=-1)) / 3.0]
    print(f"[bench] c4 check: eq36 vs eq35 {out['alpha_rel_diff_eq36_vs_eq35']:.2e}, mixed vs FP64 "
          f"{out['alpha_rel_diff_mixed_vs_fp64']:.2e}", file=sys.stderr, flush=True)
    print(json.dumps(out))


def main_c5(args):
    import numpy as np
    import torch

    from paper_2503_23144_amd import lrcc
    from paper_2503_23144_amd.synth import CONFIGS, config_inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:  # reference for the HBM byte counters: 1 GiB read, 1 GiB written
        gemm_probe(lrcc, calibrate=True, nrhs=0)
    if args.gemm_probe:
        gemm_probe(lrcc, o=40, v=400, nrhs=args.chunk, tile=0)
        return
    inp = config_inputs("c5")
    cfg = CONFIGS["c5"]
    print(f"[bench] workload c5: o={inp.o} v={inp.v} naux={inp.naux} nw={len(inp.omegas)} gap={inp.gap:.3f}",
          file=sys.stderr, flush=True)
    dev_in = resident(inp)
    nb = args.chunk
    sig = sigma_leg(lrcc, inp, dev_in, nb, args.steps, args.warmup)
    value = sig["value"]
    ladder_ms, ladder_n, ladder_fl = sig["ladder"]
    gemm_ms, gemm_n, gemm_fl = sig["gemm"]
    ladder_avg_s = ladder_ms / 1e3 / max(ladder_n, 1)
    ladder_tf = ladder_fl / max(ladder_ms / 1e3, 1e-30) / 1e12
    po_, pv_ = inp.o * (inp.o - 1) // 2, inp.v * (inp.v - 1) // 2
    ladder_tile = lrcc.gemm_tuned_tile("mixed", False, True, nb * po_, pv_, pv_, ladder=True)
    traffic = measured_traffic("c5", ladder_tile)
    po, pv = inp.o * (inp.o - 1) // 2, inp.v * (inp.v - 1) // 2
    out = {
        "metric": METRIC, "value": value, "unit": "sigma evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * sig["seconds"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "dtype_detail": "complex FP32 products (3M on FP32 MFMA, FP32 accumulation) + complex FP64 diagonal",
        "data": "synthetic",
        "config": {"workload": f"c5: o={cfg['o']} v={cfg['v']} naux={cfg['naux']} (O={po}, V={pv} packed pairs; "
                               f"W {pv * pv * 8 / 1e9:.1f} GB FP32 in HBM), batched mixed-precision right Jacobian "
                               f"products over chunks of {nb} of the 3 dipole directions x {len(cfg['omegas'])} omegas "
                               f"in [0,{max(cfg['omegas']):.1f}] Ha",
                   "precision": "mixed", "rhs_per_product": nb, "memory_layout": "lean",
                   "ring_dt1_terms": "factored (Z1 = t2 . <ov||vv>, formed once per T)",
                   "amplitudes": "seeded random T (0.01 N(0,1)) and X (N(0,1)), complex"},
        "ladder_tflops": ladder_tf,
        "ladder_complex_equiv_tflops": ladder_tf * 8.0 / 6.0,
        "gemm_all_tflops": gemm_fl / max(gemm_ms / 1e3, 1e-30) / 1e12, "gemm_all_ms_per_step": gemm_ms / args.steps,
        "gemm_launches_per_step": gemm_n / args.steps,
        "roofline": {"bound": "mfma", "achieved": ladder_tf, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                     "frac": ladder_tf / PEAK["fp32"],
                     "traffic": (traffic or {}).get("bytes_per_launch"), "traffic_unit": "bytes per launch",
                     "traffic_source": traffic,
                     "algorithmic_flops_per_launch": 6.0 * nb * po * pv * pv,
                     "kernel": "zgemm_kernel<float, false, true, 1, ...> (packed vvvv ladder, 3M)",
                     "tile": TILE_NAMES.get(ladder_tile), "avg_launch_ms": 1e3 * ladder_avg_s, "launches": ladder_n},
        "setup_s": sig["setup_s"],
    }
    if not args.no_fp64:
        fp = fp64_plain_leg(lrcc, inp, dev_in, sig["t"], sig["X0"])
        mvf = float(np.abs(sig["row0_mixed"] - fp["row0_fp64"]).max() / np.abs(fp["row0_fp64"]).max())
        out["fp64_plain"] = {k: v for k, v in fp.items() if k != "row0_fp64"}
        out["fp64_plain"]["sample"] = (f"{fp['products']} right products of one right-hand side each at o=40, v=400, "
                                       "FP64 W (102 GB) resident, ring dt1 terms factored as in the mixed leg")
        out["mixed_over_fp64_plain_sigma_rate"] = value / fp["sigma_evals_per_s"]
        out["check_mixed_vs_fp64_rel"] = mvf
        out["check_adjoint_identity_rel"] = fp["adjoint_identity_rel"]
        print(f"[bench] c5 checks: mixed vs FP64 {mvf:.2e}, adjoint identity {fp['adjoint_identity_rel']:.2e}",
              file=sys.stderr, flush=True)
        assert mvf < 2e-5 and fp["adjoint_identity_rel"] < 1e-10, "products at full size fail their checks"
    if args.solve_omegas > 1 or args.solve_range:  # a grid of frequencies, alpha per frequency group
        if args.solve_range:
            lo, hi = (int(x) for x in args.solve_range.split(":"))
            idx = np.arange(lo, hi)
        else:
            idx = np.linspace(0, len(cfg["omegas"]) - 1, args.solve_omegas).round().astype(int)
        grid = [float(cfg["omegas"][k]) for k in idx]
        out["c5_solve_grid"], _ = solve_leg(lrcc, inp, dev_in, grid, tol=args.tol, keep_response=False, eq36=False)
        out["c5_solve_grid"]["subset"] = (f"3 dipole directions x {len(grid)} of the 64 frequencies {grid}; T, "
                                          "Lambda, then X, Y and alpha (Eq. 35) one frequency at a time")
    elif not args.no_solve:
        out["c5_solve"], a35 = solve_leg(lrcc, inp, dev_in, [args.solve_omega], tol=args.tol)
        sv = out["c5_solve"]
        if args.solve_fp64:
            t = time.perf_counter()
            c = _c5_context(lrcc, inp, dev_in, "fp64", "full", tol=args.tol64, chunk=1, verbose=2)
            c.solve_ground()
            c.solve_lambda()
            c.solve_response([args.solve_omega])
            a64 = c.alpha(1)
            c.close()
            lrcc.trim_memory()
            sv["fp64_solve_s"] = time.perf_counter() - t
            sv["alpha_rel_diff_mixed_vs_fp64"] = float(np.abs(a35 - a64).max() / np.abs(a64).max())
            sv["alpha_rel_diff_mixed_vs_fp64_correlated_part"] = correlated_rel_diff(
                a35, a64, alpha_uncoupled_ref(inp.fock, inp.mu, inp.o, [args.solve_omega]))
            print(f"[bench] c5 fp64 solve: {sv['fp64_solve_s']:.1f} s, mixed vs FP64 alpha "
                  f"{sv['alpha_rel_diff_mixed_vs_fp64']:.2e}", file=sys.stderr, flush=True)
        out["c5_solve"]["subset"] = (f"3 dipole directions x 1 of the 64 frequencies (omega = {args.solve_omega} Ha); "
                                     "T, Lambda, X, Y, alpha by Eq. 35, then X(w), X(-w) and alpha by Eq. 36")
        out["c5_solve"]["response_sigma_evals_per_s"] = sv["response"]["sigma_evals"] / sv["response"]["seconds"]
    del dev_in
    lrcc.trim_memory()
    torch.cuda.empty_cache()
    if not args.no_c3:
        out["c3_full_pass"] = c3_pass(lrcc, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_scaled()
        out["cpu_baseline"]["host"] = host_info()
    print(json.dumps(out))


def c3_pass(lrcc, args):
    """The full pass at o=20, v=150: integrals, T, Lambda, 48 X and 48 Y,
    alpha, mixed precision, with the plain FP64 solver timed on two of the
    16 frequencies beside it."""
    import numpy as np
    import torch

    from paper_2503_23144_amd.synth import config_inputs
    inp = config_inputs("c3")
    dev_in = resident(inp)
    run_pass(lrcc, inp, "mixed", args.tol, dev_in=dev_in)  # warm-up (tiles of the new shapes)
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = run_pass(lrcc, inp, "mixed", args.tol, timing=True, dev_in=dev_in)
    torch.cuda.synchronize()
    d = time.perf_counter() - t
    lm, ln, lf = r["ladder"]
    out = {"workload": "c3: o=20 v=150 naux=300, 3 dipole directions x 16 omegas in [0,0.3] Ha, full pass",
           "sigma_evals_per_s": r["sigma_evals"] / d, "seconds": d, "phases_s": r["phases"],
           "response_sigma_evals_per_s": r["resp_sigma_evals"] / r["phases"]["response"],
           "ladder_tflops": lf / max(lm / 1e3, 1e-30) / 1e12, "ladder_avg_launch_ms": lm / max(ln, 1)}
    if args.fp64 in ("both", "plain"):
        sub = dataclasses.replace(inp, omegas=inp.omegas[:2])
        torch.cuda.synchronize()
        t = time.perf_counter()
        r64 = run_pass(lrcc, sub, "fp64", args.tol64, chunk=1, dev_in=dev_in)
        torch.cuda.synchronize()
        d64 = time.perf_counter() - t
        out["fp64_plain"] = {"sigma_evals_per_s": r64["sigma_evals"] / d64, "seconds": d64,
                             "response_sigma_evals_per_s": r64["resp_sigma_evals"] / r64["phases"]["response"],
                             "sample": "6 right-hand sides (2 of 16 frequencies), one per product",
                             "alpha_rel_diff_mixed_vs_this": float(np.abs(r["alpha"][:2] - r64["alpha"]).max()
                                                                   / np.abs(r64["alpha"]).max()),
                             "alpha_rel_diff_mixed_vs_this_correlated_part": correlated_rel_diff(
                                 r["alpha"][:2], r64["alpha"],
                                 alpha_uncoupled_ref(inp.fock, inp.mu, inp.o, inp.omegas[:2]))}
        out["mixed_over_fp64_plain_sigma_rate"] = out["sigma_evals_per_s"] / out["fp64_plain"]["sigma_evals_per_s"]
        out["mixed_over_fp64_plain_response_rate"] = (out["response_sigma_evals_per_s"]
                                                      / out["fp64_plain"]["response_sigma_evals_per_s"])
    print(f"[bench] c3 full pass: {d:.1f} s, {out['sigma_evals_per_s']:.1f} sigma evals/s", file=sys.stderr,
          flush=True)
    del dev_in
    lrcc.trim_memory()
    torch.cuda.empty_cache()
    return out


def main_full_pass(args):
    """The o=20, v=150 full pass as the headline (--workload c3)."""
    import numpy as np
    import torch

    from paper_2503_23144_amd import lrcc
    from paper_2503_23144_amd.synth import CONFIGS, config_inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.gemm_probe:
        gemm_probe(lrcc)
        return
    inp = config_inputs(args.workload)
    cfg = CONFIGS[args.workload]
    print(f"[bench] workload {args.workload}: o={inp.o} v={inp.v} naux={inp.naux} "
          f"nw={len(inp.omegas)} gap={inp.gap:.3f}", file=sys.stderr, flush=True)

    if args.calibrate_copy:
        src = torch.ones(2**27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("[bench] calibration copy: 1 GiB read, 1 GiB written", file=sys.stderr, flush=True)
        del src, dst
    dev_in = resident(inp)
    for w in range(args.warmup):
        r = run_pass(lrcc, inp, "mixed", args.tol, dev_in=dev_in)
        print(f"[bench] warmup {w}: sigma evals {r['sigma_evals']}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sig = 0
    last = None
    for s in range(args.steps):
        last = run_pass(lrcc, inp, "mixed", args.tol, timing=True, dev_in=dev_in)
        sig += last["sigma_evals"]
        print(f"[bench] step {s}: sigma evals {last['sigma_evals']}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = sig / dt

    po_, pv_ = cfg["o"] * (cfg["o"] - 1) // 2, cfg["v"] * (cfg["v"] - 1) // 2
    ladder_tile = lrcc.gemm_tuned_tile("mixed", False, True, 3 * len(cfg["omegas"]) * po_, pv_, pv_, ladder=True)
    traffic = measured_traffic(args.workload, ladder_tile)
    ladder_ms, ladder_n, ladder_fl = last["ladder"]
    gemm_ms, gemm_n, gemm_fl = last["gemm"]
    ladder_avg_s = ladder_ms / 1e3 / max(ladder_n, 1)
    ladder_tf = ladder_fl / max(ladder_ms / 1e3, 1e-30) / 1e12
    out = {
        "metric": METRIC, "value": value, "unit": "sigma evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64",
        "dtype_detail": "complex FP32 products (3M, FP32 MFMA) + complex FP64 residuals", "data": "synthetic",
        "config": {"workload": f"{args.workload}: o={cfg['o']} v={cfg['v']} naux={cfg['naux']}, 3 dipole directions "
                               f"x {len(cfg['omegas'])} omegas in [{min(cfg['omegas']):.2f},{max(cfg['omegas']):.2f}] Ha, "
                               "full pass (integrals, T, Lambda, X, Y, alpha)",
                   "precision": "mixed", "tol_residual": args.tol, "tol_residual_fp64": args.tol64},
        "ladder_tflops": ladder_tf,
        "ladder_complex_equiv_tflops": ladder_tf * 8.0 / 6.0,
        "gemm_all_tflops": gemm_fl / max(gemm_ms / 1e3, 1e-30) / 1e12, "gemm_all_ms": gemm_ms, "gemm_launches": gemm_n,
        "roofline": {"bound": "mfma", "achieved": ladder_tf, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                     "frac": ladder_tf / PEAK["fp32"],
                     "traffic": (traffic or {}).get("bytes_per_launch"), "traffic_unit": "bytes per launch",
                     "traffic_source": traffic,
                     "kernel": "zgemm_kernel<float, false, true, 1> (packed vvvv ladder, 3M)",
                     "avg_launch_ms": 1e3 * ladder_avg_s, "launches": ladder_n},
    }
    out["phases_s"] = last["phases"]
    out["response_sigma_evals_per_s"] = last["resp_sigma_evals"] / last["phases"]["response"]
    if args.fp64 != "none":
        # plain FP64 solver: one right-hand side per Jacobian product; and FP64 batched
        runs = [r for r in (("fp64_plain", 1), ("fp64_batched", 0)) if args.fp64 in ("both", r[0][5:])]
        for name, chunk in runs:
            # the one-RHS-per-product solver is timed on the first two
            # frequencies (6 right-hand sides); its rate is per product
            sub = inp if chunk != 1 else dataclasses.replace(inp, omegas=inp.omegas[:2])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r64 = run_pass(lrcc, sub, "fp64", args.tol64, timing=True, chunk=chunk, dev_in=dev_in)
            torch.cuda.synchronize()
            d64 = time.perf_counter() - t1
            ref_alpha = last["alpha"][: len(sub.omegas)]
            err = float(np.abs(ref_alpha - r64["alpha"]).max() / np.abs(r64["alpha"]).max())
            l64 = r64["ladder"]
            out[name] = {"sigma_evals_per_s": r64["sigma_evals"] / d64, "seconds": d64,
                         "response_sigma_evals_per_s": r64["resp_sigma_evals"] / r64["phases"]["response"],
                         "phases_s": r64["phases"],
                         "ladder_tflops": l64[2] / max(l64[0] / 1e3, 1e-30) / 1e12,
                         "alpha_rel_diff_mixed_vs_this": err,
                         "sample": f"{3 * len(sub.omegas)} right-hand sides ({len(sub.omegas)} of "
                                   f"{len(inp.omegas)} frequencies), one per product" if chunk == 1 else "full pass"}
            print(f"[bench] {name}: {d64:.1f} s", file=sys.stderr, flush=True)
        for name, _ in runs:
            out[f"mixed_over_{name}_sigma_rate"] = value / out[name]["sigma_evals_per_s"]
            if out[name]["sample"] == "full pass":
                out[f"mixed_over_{name}_time"] = out[name]["seconds"] / (dt / args.steps)
    if not args.no_eq36:
        # the same mixed pass with alpha by the Eq. 36 route: right solves at
        # +w and -w and one F X product per right-hand side instead of the
        # left (Y) solves; alpha must agree with the Eq. 35 pass
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        r36 = run_pass(lrcc, inp, "mixed", args.tol, dev_in=dev_in, quadratic=True)
        torch.cuda.synchronize()
        d36 = time.perf_counter() - t1
        out["eq36_route"] = {"sigma_evals_per_s": r36["sigma_evals"] / d36, "seconds": d36,
                             "phases_s": r36["phases"],
                             "alpha_rel_diff_vs_eq35": float(np.abs(r36["alpha"] - last["alpha"]).max()
                                                             / np.abs(last["alpha"]).max())}
        print(f"[bench] eq36 route: {d36:.1f} s", file=sys.stderr, flush=True)
    if not args.no_ladder_modes:
        # the same mixed pass without the full resident vvvv matrix: rebuilt
        # from the DF factors in every ladder contraction ("direct"), or held
        # as its upper triangle in row blocks ("triangle")
        nr = 3 * len(inp.omegas)
        out["ladder_storage"] = {}
        for mode in ("direct", "triangle"):
            run_pass(lrcc, inp, "mixed", args.tol, dev_in=dev_in, ladder=mode)  # warm-up: tiles of the new shapes
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rd = run_pass(lrcc, inp, "mixed", args.tol, timing=True, dev_in=dev_in, ladder=mode)
            torch.cuda.synchronize()
            dd = time.perf_counter() - t1
            ld = rd["ladder"]
            out["ladder_storage"][mode] = {
                "sigma_evals_per_s": rd["sigma_evals"] / dd, "seconds": dd,
                "ladder_ms": ld[0], "ladder_launches": ld[1],
                "alpha_rel_diff_vs_full_w": float(np.abs(rd["alpha"] - last["alpha"]).max()
                                                  / np.abs(last["alpha"]).max()),
                "workspace_estimate_gib": lrcc.workspace_bytes(inp.o, inp.v, inp.naux, nr, "mixed",
                                                               ladder=mode) / 2**30}
            print(f"[bench] ladder storage {mode}: {dd:.1f} s", file=sys.stderr, flush=True)
        out["ladder_storage"]["full_workspace_estimate_gib"] = lrcc.workspace_bytes(
            inp.o, inp.v, inp.naux, nr, "mixed") / 2**30
        out["ladder_storage"]["note"] = ("ladder_ms covers the ladder GEMMs (for 'direct' not the W rebuild); "
                                         "W at this size is 1 GB (FP32) + 2 GB (FP64)")
    if not args.no_truncation:
        nw = len(inp.omegas)
        out["truncation_curve"] = truncation_curve(lrcc, inp, dev_in, last["alpha"], (0, nw // 2), args.tol)
    if not args.no_ladder_scale:
        out["ladder_o40_v400"] = ladder_at_scale(lrcc)
    if not args.no_sigma_table:
        out["sigma_rates"] = sigma_rates(lrcc)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inp)
        out["cpu_baseline"]["host"] = host_info()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
