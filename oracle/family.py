"""The algorithm family of Section 2 -- TEST INFRASTRUCTURE ONLY (oracle).

Written from the paper's description, independently of the GPU library:

* Table 1 fixes, for each of the five kernels, how many contracted indices and
  how many free indices (and from which input) the kernel call keeps:
      dot   1 contracted, 0 free
      axpy  0 contracted, 1 free from exactly one input
      gemv  1 contracted, 1 free from exactly one input
      ger   0 contracted, 1 free from A and 1 free from B
      gemm  1 contracted, 1 free from A and 1 free from B
  Every other index is sliced, i.e. becomes a loop (Section 2, slicing).
* All permutations of those loops are generated (Section 2, after Table 1).
* A matrix operand of gemv, ger or gemm needs one contiguous dimension; a slice
  without one is first copied to a temporary (Section 2, before the case
  study; Algs. for Test 2 and Test 3).  The copy sits in the innermost loop the
  slice depends on.
* Names list the sliced indices in loop order, with an apostrophe after the
  loop in which a copy runs, then the kernel (Section 2, footnote on names).
* Numbering is kernel-major in the order dot, axpy, gemv, ger, gemm (the
  legends of Figures 2-7 number the case study's variants 1-36 this way).

Reading (the paper prints no general ordering rule): within a kernel, kept
index combinations are ordered with the kept free indices in C's order first,
the kept contracted index (A's order) last; loop orders are the permutations in
lexicographic order over the base order "C's indices, then the contracted
indices in A's order".  This reproduces every printed legend order.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

from . import split_spec

KERNELS = ("dot", "axpy", "gemv", "ger", "gemm")


@dataclass(frozen=True)
class Operand:
    """One kernel operand: the tensor name and, per tensor axis, either the
    index letter of a loop that fixes it or None for ':' (kept)."""
    tensor: str                 # 'A', 'B' or 'C'
    letters: str                # the tensor's spec letters
    fixed: tuple                # per axis: True if sliced (fixed by a loop)

    def pattern(self) -> str:
        return "[" + ",".join(ch if f else ":" for ch, f in zip(self.letters, self.fixed)) + "]"


@dataclass(frozen=True)
class Variant:
    number: int
    kernel: str
    kept: tuple          # kept index letters
    loops: tuple         # sliced index letters, outermost first
    copies: tuple        # ((tensor, level), ...) level = loop position the copy runs in, -1 = before all loops
    name: str
    operands: tuple = field(default=())   # (A, B, C) Operand records


def roles(spec: str):
    """Contracted indices (A's order), free indices of A and of B (C's order),
    the base order used for loop permutations."""
    sa, sb, sc = split_spec(spec)
    contracted = [ch for ch in sa if ch in sb and ch not in sc]
    free_a = [ch for ch in sc if ch in sa]
    free_b = [ch for ch in sc if ch in sb]
    base = list(sc) + contracted
    return contracted, free_a, free_b, base


def _kept_combos(kernel, contracted, free_a, free_b, free_c):
    if kernel == "dot":
        return [(k,) for k in contracted]
    if kernel == "axpy":
        return [(f,) for f in free_c]
    if kernel == "gemv":
        return [(f, k) for f in free_c for k in contracted]
    if kernel == "ger":
        return [(fa, fb) for fa in free_a for fb in free_b]
    if kernel == "gemm":
        return [(fa, fb, k) for fa in free_a for fb in free_b for k in contracted]
    raise ValueError(kernel)


def _unit_axis(letters, strides):
    """The axis letter whose stride is 1 (Fortran default: the first)."""
    if strides is None:
        return letters[0] if letters else None
    for ch, s in zip(letters, strides):
        if s == 1:
            return ch
    return None


def enumerate_family(spec: str, strides: dict | None = None):
    """All variants of the family, numbered from 1 as in the paper's legends.

    ``strides`` optionally maps 'A'/'B'/'C' to per-axis element strides; the
    copy rule then asks for a unit-stride kept axis instead of the first axis.
    """
    sa, sb, sc = split_spec(spec)
    letters = {"A": sa, "B": sb, "C": sc}
    strides = strides or {}
    contracted, free_a, free_b, base = roles(spec)
    rank = {ch: r for r, ch in enumerate(base)}
    out = []
    num = 0
    for kernel in KERNELS:
        for kept in _kept_combos(kernel, contracted, free_a, free_b, list(sc)):
            sliced = sorted((ch for ch in base if ch not in kept), key=rank.get)
            for loops in itertools.permutations(sliced):
                num += 1
                ops = []
                for t in ("A", "B", "C"):
                    ops.append(Operand(t, letters[t], tuple(ch not in kept for ch in letters[t])))
                copies = []
                for op in ops:
                    kept_axes = [ch for ch, f in zip(op.letters, op.fixed) if not f]
                    if len(kept_axes) != 2:
                        continue          # scalars and vectors take any stride
                    unit = _unit_axis(op.letters, strides.get(op.tensor))
                    if unit in kept_axes:
                        continue
                    deps = [ch for ch, f in zip(op.letters, op.fixed) if f]
                    level = max((loops.index(ch) for ch in deps), default=-1)
                    copies.append((op.tensor, level))
                name = ""
                if any(lv == -1 for _, lv in copies):
                    name += "'" * sum(1 for _, lv in copies if lv == -1)
                for pos, ch in enumerate(loops):
                    name += ch + "'" * sum(1 for _, lv in copies if lv == pos)
                name += "-" + kernel
                out.append(Variant(num, kernel, tuple(kept), tuple(loops), tuple(copies), name, tuple(ops)))
    return out


def counts(spec: str) -> dict:
    c = {k: 0 for k in KERNELS}
    for v in enumerate_family(spec):
        c[v.kernel] += 1
    c["total"] = sum(c[k] for k in KERNELS)
    return c
