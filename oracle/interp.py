"""Runs a family member as the paper's loop nest of BLAS calls -- TEST
INFRASTRUCTURE ONLY (oracle).

Each variant of ``family.enumerate_family`` is executed literally: the sliced
indices are loops in the variant's order, copies of operand slices are taken in
the loop the name marks with an apostrophe (Section 2; Algs. for Tests 2 and 3),
and the innermost statement is one of the five kernels with its BLAS meaning
(Section 2, kernel list):
    dot   alpha := x^T y          axpy  y := alpha x + y
    gemv  y := A x + y            ger   A := x y^T + A
    gemm  C := A B + C
The kernels are scalar Python loops, so this is only for tiny extents.  A copy
is taken when its loop is entered, so a copy placed in the wrong loop would
feed a stale slice to the kernel and the result would differ from the plain
contraction: running every variant checks the family, not just the arithmetic.
"""
from __future__ import annotations

import numpy as np

from . import split_spec


def _view(X, letters, fixed, env):
    idx = tuple(env[ch] if f else slice(None) for ch, f in zip(letters, fixed))
    return idx, X[idx]


def _kept(letters, fixed):
    return [ch for ch, f in zip(letters, fixed) if not f]


def run_variant(v, spec: str, extents: dict, A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Accumulate contract(A, B) into C (C += A.B) with variant ``v``."""
    sa, sb, sc = split_spec(spec)
    letters = {"A": sa, "B": sb, "C": sc}
    ops = {op.tensor: op for op in v.operands}
    arrays = {"A": A, "B": B, "C": C}
    copies_at = {}
    for t, lv in v.copies:
        copies_at.setdefault(lv, []).append(t)
    temps = {}
    env = {}

    def take_copies(level):
        for t in copies_at.get(level, []):
            op = ops[t]
            deps = [ch for ch, f in zip(op.letters, op.fixed) if f]
            for ch in deps:
                if ch not in env:
                    raise AssertionError(f"{v.name}: copy of {t} placed outside loop {ch}")
            idx, view = _view(arrays[t], op.letters, op.fixed, env)
            temps[t] = (idx, np.array(view, copy=True))

    def put_back(level):
        for t in copies_at.get(level, []):
            if t == "C":
                idx, tmp = temps["C"]
                C[idx] = tmp

    def operand(t):
        if t in temps:
            return temps[t][1]
        op = ops[t]
        return _view(arrays[t], op.letters, op.fixed, env)[1]

    def body():
        a, b = operand("A"), operand("B")
        ka, kb, kc = (_kept(letters[t], ops[t].fixed) for t in ("A", "B", "C"))
        if v.kernel == "dot":
            # C[f] += x^T y over the one kept contracted index
            k = v.kept[0]
            n = extents[k]
            s = 0.0
            for r in range(n):
                s += float(a[r]) * float(b[r])
            cidx = tuple(env[ch] for ch in sc)
            if "C" in temps:
                temps["C"][1][()] += s
            else:
                C[cidx] += s
            return
        c = operand("C")
        if v.kernel == "axpy":
            f = v.kept[0]
            if f in ka:        # y := alpha x + y with x from A, alpha from B
                x, alpha = a, float(b)
            else:
                x, alpha = b, float(a)
            for r in range(extents[f]):
                c[r] += alpha * float(x[r])
        elif v.kernel == "gemv":
            f, k = v.kept
            mat, vec = (a, b) if f in ka else (b, a)
            mat_letters = ka if f in ka else kb
            for r in range(extents[f]):
                s = 0.0
                for q in range(extents[k]):
                    ij = (r, q) if mat_letters.index(f) == 0 else (q, r)
                    s += float(mat[ij]) * float(vec[q])
                c[r] += s
        elif v.kernel == "ger":
            fa, fb = v.kept
            for r in range(extents[fa]):
                for q in range(extents[fb]):
                    ij = (r, q) if kc.index(fa) == 0 else (q, r)
                    c[ij] += float(a[r]) * float(b[q])
        elif v.kernel == "gemm":
            fa, fb, k = v.kept
            for r in range(extents[fa]):
                for q in range(extents[fb]):
                    s = 0.0
                    for p in range(extents[k]):
                        ia = (r, p) if ka.index(fa) == 0 else (p, r)
                        ib = (p, q) if kb.index(k) == 0 else (q, p)
                        s += float(a[ia]) * float(b[ib])
                    ij = (r, q) if kc.index(fa) == 0 else (q, r)
                    c[ij] += s
        else:
            raise ValueError(v.kernel)

    def level(pos):
        if pos == len(v.loops):
            body()
            return
        ch = v.loops[pos]
        for val in range(extents[ch]):
            env[ch] = val
            take_copies(pos)
            level(pos + 1)
            put_back(pos)
        del env[ch]

    take_copies(-1)
    level(0)
    put_back(-1)
    return C
