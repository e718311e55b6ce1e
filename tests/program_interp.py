"""Reference interpreter for the library's serialized operation lists.

Test infrastructure: executes, with numpy einsum on the host, exactly the
operation lists the HIP library runs on the GPU (as returned by
``lrcc_program_text``), so that the host-side derivation of the right sigma,
left sigma, xi, eta and F X programs can be checked against the oracle
without a GPU.
"""
from __future__ import annotations

import numpy as np

ADD, CONTRACT, PACK, UNPACK, ZERO = range(5)
BATCH = "Z"


def parse(text: str):
    tensors, ops = {}, []
    for line in text.splitlines():
        f = line.split()
        if not f:
            continue
        if f[0] == "T":
            tensors[int(f[1])] = dict(name=f[2], cls="" if f[3] == "-" else f[3], role=int(f[4]),
                                      batched=bool(int(f[5])))
        elif f[0] == "O":
            d = lambda s: "" if s == "-" else s
            ops.append(dict(kind=int(f[1]), acc=bool(int(f[2])), alpha=complex(float(f[3]), float(f[4])),
                            out=int(f[5]), oi=d(f[6]), a=int(f[7]), ai=d(f[8]), b=int(f[9]), bi=d(f[10]),
                            m=(int(f[11]), int(f[12]))))
    return tensors, ops


def pairs(n):
    p0, p1 = [], []
    for b in range(n):
        for a in range(b):
            p0.append(a)
            p1.append(b)
    return np.array(p0, dtype=np.int64), np.array(p1, dtype=np.int64)


def _pack_pair(x, axis, mode):
    n = x.shape[axis]
    p0, p1 = pairs(n)
    xm = np.moveaxis(x, (axis, axis + 1), (-2, -1))
    y = xm[..., p0, p1]
    if mode:
        y = y - xm[..., p1, p0]
    return np.moveaxis(y, -1, axis)


def _unpack_pair(y, axis, mode, n):
    p0, p1 = pairs(n)
    ym = np.moveaxis(y, axis, -1)
    x = np.zeros(ym.shape[:-1] + (n, n), dtype=y.dtype)
    x[..., p0, p1] = ym
    if mode:
        x[..., p1, p0] = -ym
    return np.moveaxis(x, (-2, -1), (axis, axis + 1))


def _align(packed: str, full: str):
    """Positions in `full` of each packed-pair letter of `packed`."""
    out, p = [], 0
    for ch in packed:
        if p < len(full) and full[p] == ch:
            p += 1
        else:
            out.append(p)
            p += 2
    assert p == len(full), (packed, full)
    return out


class Interp:
    def __init__(self, tensors, o, v, nb):
        self.t, self.o, self.v, self.nb = tensors, o, v, nb
        self.dim = {"o": o, "v": v, "O": o * (o - 1) // 2, "V": v * (v - 1) // 2}

    def shape(self, tid):
        s = tuple(self.dim[c] for c in self.t[tid]["cls"])
        return ((self.nb,) + s) if self.t[tid]["batched"] else s

    def id(self, name):
        for k, d in self.t.items():
            if d["name"] == name:
                return k
        raise KeyError(name)

    def run(self, ops, env):
        for op in ops:
            out = op["out"]
            ob = self.t[out]["batched"]
            if op["kind"] == ZERO:
                env[out] = np.zeros(self.shape(out), dtype=np.complex128)
                continue
            a = env[op["a"]]
            ab = self.t[op["a"]]["batched"]
            if op["kind"] == CONTRACT:
                b = env[op["b"]]
                bb = self.t[op["b"]]["batched"]
                sub = f"{BATCH if ab else ''}{op['ai']},{BATCH if bb else ''}{op['bi']}->{BATCH if ob else ''}{op['oi']}"
                val = np.einsum(sub, a, b)
            elif op["kind"] == ADD:
                sub = f"{BATCH if ab else ''}{op['ai']}->{BATCH if ob else ''}{op['oi']}"
                val = np.einsum(sub, a)
            elif op["kind"] == PACK:
                pos = _align(op["oi"], op["ai"])
                val = a
                for k in reversed(range(len(pos))):
                    val = _pack_pair(val, pos[k] + (1 if ab else 0), op["m"][k])
            else:  # UNPACK
                pos = _align(op["ai"], op["oi"])
                val = a
                full = op["oi"]
                for k in reversed(range(len(pos))):
                    # the packed letter sits at (its index in ai) in the current array
                    n = self.dim[{"o": "o", "v": "v"}[_cls(full[pos[k]])]]
                    val = _unpack_pair(val, _packed_axis(op["ai"], full, k) + (1 if ab else 0), op["m"][k], n)
            val = op["alpha"] * val
            if op["acc"]:
                env[out] = env[out] + val
            else:
                env[out] = np.array(val, dtype=np.complex128).reshape(self.shape(out))
        return env


def executor_order(ops):
    """The order in which the executor runs `ops`: within each run of ADD ops
    it groups the ops by output tensor (each group keeping its order, groups
    in the order of their first op) when no op of the run reads a tensor that
    another op of the run writes and no tensor is first written after the
    run's first op; otherwise it keeps the list order.  Mirrors the grouping
    rule of the executor's summed permutes."""
    out, i = [], 0
    while i < len(ops):
        if ops[i]["kind"] != ADD:
            out.append(ops[i])
            i += 1
            continue
        w = i
        while w < len(ops) and ops[w]["kind"] == ADD:
            w += 1
        regroup = w - i >= 2
        for k in range(i, w):
            if any(q != k and ops[k]["a"] == ops[q]["out"] for q in range(i, w)):
                regroup = False
            if k > i and not any(ops[q]["out"] == ops[k]["out"] for q in range(k)):
                regroup = False
        run = ops[i:w]
        if regroup:
            heads = []
            for op in run:
                if op["out"] not in heads:
                    heads.append(op["out"])
            run = [op for h in heads for op in run if op["out"] == h]
        out.extend(run)
        i = w
    return out


def _cls(ch):
    return "o" if "i" <= ch <= "n" else "v"


def _packed_axis(packed: str, full: str, k: int):
    """Axis in `packed` of its k-th packed-pair letter."""
    cnt, p = 0, 0
    for ax, ch in enumerate(packed):
        if p < len(full) and full[p] == ch:
            p += 1
        else:
            if cnt == k:
                return ax
            cnt += 1
            p += 2
    raise ValueError


def blocks_from_df(B, o):
    """The integral blocks the library's residual program declares, built
    here independently from the density-fitting factors."""
    B = np.asarray(B)
    v = B.shape[1] - o
    sl = {"o": slice(0, o), "v": slice(o, None)}

    def blk(spec):
        P, Q, R, S = (sl[c] for c in spec)
        return np.einsum("xpr,xqs->pqrs", B[:, P, R], B[:, Q, S]) - np.einsum("xps,xqr->pqrs", B[:, P, S], B[:, Q, R])

    a0, a1 = pairs(v)
    out = {k: blk(k) for k in ["oooo", "ooov", "oovv", "ovvo", "ovvv", "vvoo", "vvvo", "ovoo"]}
    vvvv = blk("vvvv")
    out["W"] = vvvv[a0[:, None], a1[:, None], a0[None, :], a1[None, :]]
    out["govvp"] = out["ovvv"][:, :, a0, a1]
    return {("g" + k if k not in ("W", "govvp") else k): val for k, val in out.items()}


def fock_blocks(F, o):
    F = np.asarray(F)
    return {"foo": F[:o, :o], "fov": F[:o, o:], "fvo": F[o:, :o], "fvv": F[o:, o:]}
