"""Split-precision contraction -- TEST INFRASTRUCTURE ONLY (oracle).

The precision form computes the contraction with low-precision matrix
products and wins the accuracy back as follows (the reading used throughout):

  1. Per-slice power-of-two scaling.  A slice is the sub-tensor at one fixed
     value of all free indices of an operand (A[:, a, :] for A_iaj).  Its
     exponent is e = floor(log2(max |x|)) (0 for an all-zero slice) and the
     slice is multiplied by 2**-e, which is exact.
  2. Three-term split of every scaled entry x by round-to-nearest-even to a
     format with p significant bits (BF16: p = 8; OCP FP8 E4M3: p = 4):
         t1 = rn(x),  r1 = x - t1,  t2 = rn(r1),  t3 = rn(r1 - t2)
     The residuals are exact in FP64.
  3. The products t_A,p * t_B,q with p + q <= 4 (six of the nine) are summed.
  4. The sum is multiplied by 2**(e_A + e_B) of the two slices.

This module forms step 3 in FP64 (the plain loop-nest oracle on the term
tensors), so it is the split method with exact accumulation; the GPU
accumulates in FP32 over K chunks and combines chunks in FP64, and the tests
bound that difference.  The FP8 form scales the p-th term by 2**(4(p-1)) before
rounding so every term stays inside E4M3's normal range; that scale is undone
after the product.
"""
from __future__ import annotations

import numpy as np

from . import contract as _contract, split_spec

BF16_BITS = 8       # significand bits including the implicit one
E4M3_BITS = 4
E4M3_MAX = 448.0
E4M3_MIN_NORMAL_EXP = -6

PAIRS = [(p, q) for p in (1, 2, 3) for q in (1, 2, 3) if p + q <= 4]


def round_bits(x: np.ndarray, bits: int) -> np.ndarray:
    """Round-to-nearest-even of FP64 values to `bits` significant bits with an
    unbounded exponent range: x = m * 2**E with 0.5 <= |m| < 1 (frexp), keep
    rint(m * 2**bits) (numpy's rint rounds halves to even)."""
    x = np.asarray(x, dtype=np.float64)
    m, E = np.frexp(x)
    return np.ldexp(np.rint(np.ldexp(m, bits)), E - bits)


def round_e4m3(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even to OCP FP8 E4M3 (4 significant bits, smallest
    normal 2**-6, subnormal spacing 2**-9, largest finite 448; values beyond
    are saturated to +-448)."""
    x = np.asarray(x, dtype=np.float64)
    m, E = np.frexp(x)
    # exponent of the leading bit is E-1; below the normal range the spacing is fixed at 2**-9
    lead = np.maximum(E - 1, E4M3_MIN_NORMAL_EXP)
    q = np.ldexp(np.rint(np.ldexp(x, -(lead - (E4M3_BITS - 1)))), lead - (E4M3_BITS - 1))
    return np.clip(q, -E4M3_MAX, E4M3_MAX)


def slice_exponents(X: np.ndarray, letters: str, free: str) -> np.ndarray:
    """floor(log2(max |X|)) over every slice at fixed free indices; shape = the
    free axes in `letters` order.  All-zero slices get 0."""
    axes = tuple(ax for ax, ch in enumerate(letters) if ch not in free)
    amax = np.max(np.abs(X), axis=axes) if axes else np.abs(X)
    with np.errstate(divide="ignore"):
        _, E = np.frexp(amax)
    e = (E - 1).astype(np.int64)
    return np.where(amax > 0, e, 0)


def _broadcast(e: np.ndarray, src: str, dst: str, free: str) -> np.ndarray:
    """Exponents with axes = the free letters in `src` order, laid out for an
    array whose axes are the letters of `dst` (size-1 axes elsewhere)."""
    src_free = [ch for ch in src if ch in free]
    dst_free = [ch for ch in dst if ch in free]
    e = np.transpose(e, [src_free.index(ch) for ch in dst_free]) if len(src_free) > 1 else e
    shape = [1] * len(dst)
    j = 0
    for ax, ch in enumerate(dst):
        if ch in free:
            shape[ax] = e.shape[j]
            j += 1
    return e.reshape(shape)


def split_terms(X: np.ndarray, letters: str, free: str, kind: str = "bf16"):
    """Scaled three-term split of operand X; returns (terms[3], exponents)."""
    e = slice_exponents(X, letters, free)
    xs = np.ldexp(X, -_broadcast(e, letters, letters, free))
    if kind == "bf16":
        rn = lambda v: round_bits(v, BF16_BITS)
        t1 = rn(xs)
        r1 = xs - t1
        t2 = rn(r1)
        t3 = rn(r1 - t2)
    elif kind == "fp8":
        # term p carries an extra 2**(4(p-1)) so that it stays in E4M3's normal range
        t1 = round_e4m3(xs)
        r1 = xs - t1
        t2 = np.ldexp(round_e4m3(np.ldexp(r1, 4)), -4)
        t3 = np.ldexp(round_e4m3(np.ldexp(r1 - t2, 8)), -8)
    else:
        raise ValueError(kind)
    return [np.array(t, order="F") for t in (t1, t2, t3)], e


def contract_split(spec: str, extents: dict, A: np.ndarray, B: np.ndarray, kind: str = "bf16",
                   pairs=PAIRS, C: np.ndarray | None = None, alpha: float = 1.0, beta: float = 0.0):
    """The split contraction with exact (FP64) accumulation of the products."""
    sa, sb, sc = split_spec(spec)
    fa = "".join(ch for ch in sa if ch in sc)
    fb = "".join(ch for ch in sb if ch in sc)
    TA, eA = split_terms(A, sa, fa, kind)
    TB, eB = split_terms(B, sb, fb, kind)
    acc = np.zeros([extents[ch] for ch in sc], order="F")
    for p, q in pairs:
        acc += _contract(spec, extents, TA[p - 1], TB[q - 1])
    # 2**(eA + eB) on C's axes
    scale = np.zeros([extents[ch] for ch in sc], dtype=np.int64)
    scale += _broadcast(eA, sa, sc, fa) if fa else 0
    scale += _broadcast(eB, sb, sc, fb) if fb else 0
    out = alpha * np.ldexp(acc, scale)
    if beta != 0.0:
        out = out + beta * C
    return np.array(out, order="F")
