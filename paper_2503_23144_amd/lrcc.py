"""ctypes binding of liblrcc.so (include/lrcc.h).

Argument marshalling only: every computation runs in the HIP library.  Buffers
may be numpy arrays (host) or torch tensors (host or device); complex data
are complex128 (complex64 for the FP32 GEMM entry point).  Importing this
module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# LRCC_LIBRARY names another build of the library (e.g. the host-sanitized
# one that the host-side checks run against)
LIB_PATH = os.environ.get("LRCC_LIBRARY") or os.path.join(HERE, "liblrcc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lrcc.h")

OK, E_INVALID, E_STATE, E_NOMEM, E_HIP, E_NOCONV, E_SINGULAR, E_INTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
HOST, DEVICE = 0, 1
FP64, MIXED = 0, 1
SIDE_RESIDUAL, SIDE_RIGHT, SIDE_LEFT = 0, 1, 2
AMP_T, AMP_LAMBDA, AMP_X, AMP_Y, AMP_XMINUS = 0, 1, 2, 3, 4
(PROG_RESIDUAL, PROG_RIGHT, PROG_LEFT, PROG_XI, PROG_HVP, PROG_ETA0, PROG_GRADL, PROG_FX, PROG_FNSPP,
 PROG_RING_SETUP, PROG_RIGHT_F, PROG_LEFT_F) = range(12)

# torch ships its own libamdhip64.so.7; load it first so that torch (device
# memory, streams) and this library share one HIP runtime in the process.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2503_23144_amd.build`")
lib = ctypes.CDLL(LIB_PATH)


class LrccError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lrcc error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("precision", ctypes.c_int),
                ("tol_residual", ctypes.c_double), ("maxit", ctypes.c_int), ("diis_size", ctypes.c_int),
                ("rhs_chunk", ctypes.c_int), ("autotune", ctypes.c_int), ("verbose", ctypes.c_int),
                ("graphs", ctypes.c_int), ("ladder_mode", ctypes.c_int), ("ladder_mode_fp64", ctypes.c_int),
                ("memory_mode", ctypes.c_int), ("ring_factored", ctypes.c_int), ("keep_response", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("sigma_evals", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp, _i, _i64, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
_sig = {
    "lrcc_default_config": (None, [ctypes.POINTER(Config)]),
    "lrcc_create": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(Config)]),
    "lrcc_destroy": (None, [_vp]),
    "lrcc_last_error": (ctypes.c_char_p, [_vp]),
    "lrcc_load_df": (_i, [_vp, _i, _i, _i, _vp, _i]),
    "lrcc_load_fock": (_i, [_vp, _vp, _i]),
    "lrcc_load_dipoles": (_i, [_vp, _i, _vp, _i]),
    "lrcc_fnspp_truncate": (_i, [_vp, _vp, _i, _d, _i, ctypes.POINTER(_i), _vp]),
    "lrcc_fns_truncate": (_i, [_vp, _d, _i, ctypes.POINTER(_i), _vp]),
    "lrcc_solve_ground": (_i, [_vp, _vp, ctypes.POINTER(Stats)]),
    "lrcc_solve_lambda": (_i, [_vp, ctypes.POINTER(Stats)]),
    "lrcc_solve_response": (_i, [_vp, _i, _vp, _vp]),
    "lrcc_solve_response_quadratic": (_i, [_vp, _i, _vp, _vp]),
    "lrcc_mp2_response": (_i, [_vp, _i, _vp, _vp, _vp, _i]),
    "lrcc_get_alpha": (_i, [_vp, _vp, _i]),
    "lrcc_sigma": (_i, [_vp, _i, _i, _vp, _vp, _vp, _i, _i]),
    "lrcc_amplitude_length": (_i64, [_vp]),
    "lrcc_get_amplitudes": (_i, [_vp, _i, _i, _vp, _i]),
    "lrcc_set_amplitudes": (_i, [_vp, _i, _i, _vp, _i]),
    "lrcc_gemm": (_i, [_i, _i, _i, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp]),
    "lrcc_gemm_noalloc": (_i, [_i, _i, _i, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _vp, _i64, _vp]),
    "lrcc_gemm_set_tile": (_i, [_i]),
    "lrcc_gemm_tuned_tile": (_i, [_i, _i, _i, _i64, _i64, _i64, _i]),
    "lrcc_program_text": (_i64, [_i, ctypes.c_char_p, _i64]),
    "lrcc_kernel_time": (_i, [_vp, _i, ctypes.POINTER(_d), ctypes.POINTER(_i64), ctypes.POINTER(_d)]),
    "lrcc_set_timing": (_i, [_vp, _i]),
    "lrcc_graph_stats": (_i, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "lrcc_trim_memory": (_i, []),
    "lrcc_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config), _i, _i, _i, _i]),
    "lrcc_set_workspace": (_i, [_vp, _vp, ctypes.c_size_t]),
    "lrcc_workspace_peak": (ctypes.c_size_t, [_vp]),
    "lrcc_build_info": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def declared_symbols():
    """Function names declared in include/lrcc.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lrcc_\w+)\s*\(", txt, flags=re.M)))


def _buf(x, dtype=np.complex128):
    """(pointer, where, keepalive) for a numpy array or torch tensor."""
    try:
        import torch
        if isinstance(x, torch.Tensor):
            if not x.is_contiguous():
                raise ValueError("tensor must be contiguous")
            return x.data_ptr(), (DEVICE if x.is_cuda else HOST), x
    except ImportError:
        pass
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, HOST, a


def program_text(which: int) -> str:
    n = lib.lrcc_program_text(which, None, 0)
    if n < 0:
        raise LrccError(E_INVALID, f"no program {which}")
    buf = ctypes.create_string_buffer(n + 1)
    lib.lrcc_program_text(which, buf, n + 1)
    return buf.value.decode()


def build_info() -> str:
    return lib.lrcc_build_info().decode()


LADDER_FULL, LADDER_DIRECT, LADDER_TRIANGLE = 0, 1, 2


def workspace_bytes(o, v, naux, nrhs, precision="fp64", diis=8, ladder="full", ladder_fp64=None, memory="auto",
                    ring_factored=None):
    """Device bytes of the whole pipeline with batches of up to nrhs
    right-hand sides (lrcc_workspace_bytes)."""
    cfg = Config()
    lib.lrcc_default_config(ctypes.byref(cfg))
    cfg.precision = {"fp64": FP64, "mixed": MIXED}[precision]
    cfg.diis_size = diis
    modes = {"full": LADDER_FULL, "direct": LADDER_DIRECT, "triangle": LADDER_TRIANGLE}
    cfg.ladder_mode = modes[ladder]
    cfg.ladder_mode_fp64 = -1 if ladder_fp64 is None else modes[ladder_fp64]
    cfg.memory_mode = {"auto": 0, "resident": 1, "lean": 2}[memory]
    cfg.ring_factored = -1 if ring_factored is None else int(bool(ring_factored))
    return int(lib.lrcc_workspace_bytes(ctypes.byref(cfg), o, v, naux, nrhs))


def trim_memory():
    """Return the device memory the library keeps for reuse (see
    lrcc_trim_memory) to the device."""
    rc = lib.lrcc_trim_memory()
    if rc != OK:
        raise LrccError(rc, lib.lrcc_last_error(None).decode())


def gemm(A, B, C, transa=False, transb=False, alpha=1.0, beta=0.0, stream=None, noalloc=False):
    """C = alpha op(A) op(B) + beta C on contiguous 2-D device tensors
    (complex128: FP64 path; complex64: FP32 3M path).  noalloc=True calls
    lrcc_gemm_noalloc (no device allocation; split-K partials in the
    library's static scratch)."""
    import torch
    prec = FP64 if A.dtype == torch.complex128 else MIXED
    m = A.shape[1] if transa else A.shape[0]
    k = A.shape[0] if transa else A.shape[1]
    n = B.shape[0] if transb else B.shape[1]
    al = (ctypes.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (ctypes.c_double * 2)(complex(beta).real, complex(beta).imag)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    fn = lib.lrcc_gemm_noalloc if noalloc else lib.lrcc_gemm
    rc = fn(prec, int(transa), int(transb), m, n, k, al, A.data_ptr(), A.shape[1], B.data_ptr(),
            B.shape[1], be, C.data_ptr(), C.shape[1], stream)
    if rc != OK:
        raise LrccError(rc, lib.lrcc_last_error(None).decode())
    return C


def gemm_tuned_tile(precision, ta, tb, m, n, k, ladder=False):
    """Tile the autotuner chose for a product shape in this process (-1: not
    timed); see lrcc_gemm_tuned_tile."""
    return int(lib.lrcc_gemm_tuned_tile({"fp64": FP64, "mixed": MIXED}[precision], int(ta), int(tb), m, n, k,
                                        int(ladder)))


def gemm_set_tile(tile):
    """Force the GEMM workgroup tile (0..4) of later launches; -1 restores
    the automatic choice."""
    rc = lib.lrcc_gemm_set_tile(int(tile))
    if rc != OK:
        raise LrccError(rc, lib.lrcc_last_error(None).decode())


class Context:
    """One system on one GPU: integrals, Fock and dipole matrices, and the
    T, Lambda, X, Y solves of LR-CCSD."""

    def __init__(self, device=0, stream=None, precision="fp64", tol=1e-10, maxit=100, diis=8, rhs_chunk=0,
                 verbose=0, autotune=True, graphs=None, ladder="full", ladder_fp64=None, memory="auto",
                 ring_factored=None, keep_response=True):
        cfg = Config()
        lib.lrcc_default_config(ctypes.byref(cfg))
        cfg.device = device
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        cfg.stream = stream
        cfg.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        cfg.tol_residual = tol
        cfg.maxit = maxit
        cfg.diis_size = diis
        cfg.rhs_chunk = rhs_chunk
        cfg.autotune = int(autotune)
        cfg.verbose = verbose
        if graphs is not None:  # else the library default (LRCC_GRAPHS)
            cfg.graphs = int(graphs)
        # storage of the vvvv matrix: "full", "direct" (rebuilt from the DF
        # factors in every ladder) or "triangle" (upper triangle only)
        modes = {"full": LADDER_FULL, "direct": LADDER_DIRECT, "triangle": LADDER_TRIANGLE}
        cfg.ladder_mode = modes[ladder]
        # W of the FP64 products in mixed precision (None: as `ladder`)
        cfg.ladder_mode_fp64 = -1 if ladder_fp64 is None else modes[ladder_fp64]
        # "auto", "resident" (dense integral blocks) or "lean" (packed / formed on use)
        cfg.memory_mode = {"auto": 0, "resident": 1, "lean": 2}[memory]
        # the dt1 part of the ring term through Z1, Z2 (None: automatic)
        cfg.ring_factored = -1 if ring_factored is None else int(bool(ring_factored))
        # False: alpha per frequency group, only the last group's X and Y kept
        cfg.keep_response = int(bool(keep_response))
        h = _vp()
        rc = lib.lrcc_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc != OK:
            raise LrccError(rc, lib.lrcc_last_error(None).decode())
        self._h = h
        self.o = self.v = self.ncomp = 0

    def close(self):
        if getattr(self, "_h", None):
            lib.lrcc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            raise LrccError(rc, lib.lrcc_last_error(self._h).decode())
        return rc

    @property
    def n(self) -> int:
        return int(lib.lrcc_amplitude_length(self._h))

    def load_df(self, o, v, B):
        p, w, keep = _buf(B)
        self._check(lib.lrcc_load_df(self._h, o, v, B.shape[0], p, w))
        self.o, self.v = o, v

    def load_fock(self, F):
        p, w, keep = _buf(F)
        self._check(lib.lrcc_load_fock(self._h, p, w))

    def load_dipoles(self, mu):
        p, w, keep = _buf(mu)
        self._check(lib.lrcc_load_dipoles(self._h, mu.shape[0], p, w))
        self.ncomp = mu.shape[0]

    def fnspp_truncate(self, omegas, thresh=1e-5, keep=0):
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        nv = ctypes.c_int()
        occ = np.zeros(self.v, dtype=np.float64)
        self._check(lib.lrcc_fnspp_truncate(self._h, om.ctypes.data, om.size, thresh, keep, ctypes.byref(nv),
                                            occ.ctypes.data))
        self.v = nv.value
        return nv.value, occ

    def fns_truncate(self, thresh=1e-5, keep=0):
        """Ground-state natural spinors (FNS, Eq. 40)."""
        nv = ctypes.c_int()
        occ = np.zeros(self.v, dtype=np.float64)
        self._check(lib.lrcc_fns_truncate(self._h, thresh, keep, ctypes.byref(nv), occ.ctypes.data))
        self.v = nv.value
        return nv.value, occ

    def solve_ground(self):
        e = (ctypes.c_double * 2)()
        s = Stats()
        self._check(lib.lrcc_solve_ground(self._h, e, ctypes.byref(s)))
        return complex(e[0], e[1]), s.as_dict()

    def solve_lambda(self):
        s = Stats()
        self._check(lib.lrcc_solve_lambda(self._h, ctypes.byref(s)))
        return s.as_dict()

    def solve_response(self, omegas, allow_noconv=False, quadratic=False):
        """X and Y solves and alpha by Eq. 35; quadratic=True takes the Eq. 36
        route (X(w) and X(-w), no Y)."""
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        st = (Stats * (2 * om.size * self.ncomp))()
        fn = lib.lrcc_solve_response_quadratic if quadratic else lib.lrcc_solve_response
        self._check(fn(self._h, om.size, om.ctypes.data, st), allow=(E_NOCONV,) if allow_noconv else ())
        return [s.as_dict() for s in st]

    def mp2_response(self, omegas):
        """(E_MP2, alpha_MP2 [nw, ncomp, ncomp]) in the current virtual space:
        the terms of the FNS++ corrections (full minus truncated space)."""
        om = np.ascontiguousarray(omegas, dtype=np.float64)
        e = (ctypes.c_double * 2)()
        out = np.zeros((om.size, self.ncomp, self.ncomp), dtype=np.complex128)
        self._check(lib.lrcc_mp2_response(self._h, om.size, om.ctypes.data, e, out.ctypes.data, HOST))
        return complex(e[0], e[1]), out

    def alpha(self, nw):
        out = np.zeros((nw, self.ncomp, self.ncomp), dtype=np.complex128)
        self._check(lib.lrcc_get_alpha(self._h, out.ctypes.data, HOST))
        return out

    def sigma(self, side, X, shifts=None, precision="fp64", out=None):
        """side: 'residual', 'right' or 'left'.  X: [nvec, n] (numpy or torch)."""
        sd = {"residual": SIDE_RESIDUAL, "right": SIDE_RIGHT, "left": SIDE_LEFT}[side]
        nvec = 1 if X.ndim == 1 else X.shape[0]
        p, w, keep = _buf(X)
        if out is None:
            if w == DEVICE:
                import torch
                out = torch.empty_like(X)
            else:
                out = np.zeros(X.shape, dtype=np.complex128)
        q, w2, keep2 = _buf(out)
        assert w2 == w, "input and output must live in the same place"
        sh = None
        if shifts is not None:
            sh = np.ascontiguousarray(shifts, dtype=np.float64)
        self._check(lib.lrcc_sigma(self._h, sd, nvec, None if sh is None else sh.ctypes.data, p, q, w,
                                   {"fp64": FP64, "mixed": MIXED}[precision]))
        return out

    def get_amplitudes(self, which, idx=0):
        out = np.zeros(self.n, dtype=np.complex128)
        self._check(lib.lrcc_get_amplitudes(self._h, which, idx, out.ctypes.data, HOST))
        return out

    def set_amplitudes(self, which, x, idx=0):
        p, w, keep = _buf(x)
        self._check(lib.lrcc_set_amplitudes(self._h, which, idx, p, w))

    def set_timing(self, on=True):
        self._check(lib.lrcc_set_timing(self._h, int(on)))

    def kernel_time(self, cls):
        ms, ln, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        self._check(lib.lrcc_kernel_time(self._h, cls, ctypes.byref(ms), ctypes.byref(ln), ctypes.byref(fl)))
        return ms.value, ln.value, fl.value

    def set_workspace(self, buf):
        """Carve every device allocation of this context from `buf` (a device
        tensor the caller keeps alive until close()); before load_df."""
        self._workspace = buf
        self._check(lib.lrcc_set_workspace(self._h, buf.data_ptr(), buf.numel() * buf.element_size()))

    def workspace_peak(self):
        return int(lib.lrcc_workspace_peak(self._h))

    def graph_stats(self):
        """(program runs captured into HIP graphs, graph replays)."""
        cap, rep = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib.lrcc_graph_stats(self._h, ctypes.byref(cap), ctypes.byref(rep)))
        return cap.value, rep.value


class RightSigma(torch.autograd.Function):
    """y = A x + s x: the CC Jacobian (Eq. 30) at the context's T applied to
    complex128 amplitude vectors x [nvec, n] (device or host).  The backward
    pass is the library's left product (the exact transpose): for a
    holomorphic map PyTorch expects grad_x = conj(A^T conj(grad_y))."""

    @staticmethod
    def forward(ctx, x, context, shifts=None, precision="fp64"):
        ctx.context, ctx.shifts, ctx.precision = context, shifts, precision
        return context.sigma("right", x.detach().contiguous(), shifts=shifts, precision=precision)

    @staticmethod
    def backward(ctx, g):
        gl = ctx.context.sigma("left", g.conj().resolve_conj().contiguous(), shifts=ctx.shifts,
                               precision=ctx.precision)
        return gl.conj().resolve_conj(), None, None, None


def right_sigma(x, context, shifts=None, precision="fp64"):
    """Differentiable A x (see RightSigma)."""
    return RightSigma.apply(x, context, shifts, precision)
