"""Oracle for the tensor-contraction library -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports it, and it
imports nothing from the GPU library: the two share no code.

Contents
  contract.c    plain FP64 loop nest (Section 1, Tensor Notation), own parser;
                batch indices (in A, B and C) and trace indices (one input
                only) read as the same sum over every index absent from C;
                the same loops over complex numbers (real and imaginary
                parts in FP64, products written out)
  family.py     the algorithm family of Section 2 (Table 1 rules x loop orders)
  interp.py     executes each family member as the paper's loops of BLAS calls
  access.py     the symbolic prediction steps of Section 3 (access distance,
                setup lists, prefetching, prefetch failures, first iterations)
  split.py      the split-precision product form (power-of-two scaled slices,
                3-term BF16 / FP8 split, compensated FP64 combine)

``contract()`` below wraps ``contract.c`` for numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "contract.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile contract.c with gcc (-O2, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-fopenmp",
                               "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_contract.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i64p, ctypes.c_int,
                                        dp, i64p, dp, i64p, dp, i64p,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_int]
        lib.oracle_contract.restype = ctypes.c_int
        lib.oracle_contract_z.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i64p, ctypes.c_int,
                                          dp, i64p, dp, i64p, dp, i64p,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        lib.oracle_contract_z.restype = ctypes.c_int
        lib.oracle_contract_par.argtypes = lib.oracle_contract.argtypes
        lib.oracle_contract_par.restype = ctypes.c_int
        _lib = lib
    return _lib


def split_spec(spec: str):
    """'abc=ai,ibc' -> ('ai', 'ibc', 'abc')."""
    out, ins = spec.split("=")
    a, b = ins.split(",")
    return a, b, out


def _elem_strides(x: np.ndarray):
    st = [s // x.itemsize for s in x.strides]
    if any(s < 0 for s in st) or any(s * x.itemsize != t for s, t in zip(st, x.strides)):
        raise ValueError("oracle: operand strides must be non-negative whole elements")
    return (ctypes.c_int64 * max(1, len(st)))(*st)


def contract(spec: str, extents: dict, A: np.ndarray, B: np.ndarray, C: np.ndarray | None = None,
             alpha: float = 1.0, beta: float = 0.0, dot2: bool = False, threads: int = 1) -> np.ndarray:
    """C = alpha * contract(A, B) + beta * C in FP64 (Section 1 definition).

    ``A``, ``B`` (and ``C``) are float64 numpy arrays whose axes follow the
    operand's spec letters, or all complex128 for the same sum over complex
    numbers (then alpha and beta may be complex); any non-negative strides are honoured, so a
    Fortran-ordered array is the paper's storage.  If ``C`` is None a new
    Fortran-ordered array is returned (beta must then be 0).  With ``dot2`` the
    sum is accumulated in doubled working precision.  ``threads`` > 1 spreads
    C's outermost index over host threads (real operands; same result bit for
    bit: each element is summed by one thread in the same order).
    """
    sa, sb, sc = split_spec(spec)
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B) or (C is not None and np.iscomplexobj(C))
    want = np.complex128 if cplx else np.float64
    for name, x, s in (("A", A, sa), ("B", B, sb)):
        if x.dtype != want:
            raise TypeError(f"oracle: {name} must be {np.dtype(want).name} (widen narrower types exactly first)")
        if x.ndim != len(s):
            raise ValueError(f"oracle: {name} has {x.ndim} axes, spec wants {len(s)}")
        for ch, n in zip(s, x.shape):
            if extents[ch] != n:
                raise ValueError(f"oracle: {name} axis {ch} is {n}, extent is {extents[ch]}")
    if C is None:
        if beta != 0.0:
            raise ValueError("oracle: beta != 0 needs an input C")
        C = np.zeros([extents[ch] for ch in sc], dtype=want, order="F")
    elif C.dtype != want:
        raise TypeError(f"oracle: C must be {np.dtype(want).name}")
    chars = "".join(sorted(extents))
    ext = (ctypes.c_int64 * len(chars))(*[int(extents[ch]) for ch in chars])
    dp = ctypes.POINTER(ctypes.c_double)
    args = (spec.encode(), chars.encode(), ext, len(chars),
            A.ctypes.data_as(dp), _elem_strides(A), B.ctypes.data_as(dp), _elem_strides(B),
            C.ctypes.data_as(dp), _elem_strides(C))
    if cplx:
        if dot2:
            raise ValueError("oracle: doubled-precision sums are for real operands")
        al, be = complex(alpha), complex(beta)
        rc = _load().oracle_contract_z(*args, al.real, al.imag, be.real, be.imag)
    elif threads > 1:
        if dot2:
            raise ValueError("oracle: doubled-precision sums run on one thread")
        rc = _load().oracle_contract_par(*args, float(alpha), float(beta), int(threads))
    else:
        rc = _load().oracle_contract(*args, float(alpha), float(beta), 1 if dot2 else 0)
    if rc != 0:
        raise ValueError(f"oracle_contract failed with code {rc} for spec {spec!r}")
    return C


def flops(spec: str, extents: dict) -> int:
    """Useful flops of a contraction: 2 * product of all extents (one multiply and
    one add per term of the defining sum)."""
    n = 1
    for ch in set(spec.replace("=", "").replace(",", "")):
        n *= int(extents[ch])
    return 2 * n


def normwise_rel_err(C_hat: np.ndarray, C_ref: np.ndarray, scale_ref: np.ndarray | None = None) -> float:
    """Frobenius-norm relative error ||C_hat - C_ref||_F / ||C_ref||_F.  When the
    reference is all zero, ``scale_ref`` (|A|.|B| contracted) is the denominator."""
    C_hat = np.asarray(C_hat)
    d = np.linalg.norm((C_hat.astype(np.result_type(C_hat, np.float64)) - C_ref).ravel())
    n = np.linalg.norm(np.asarray(C_ref).ravel())
    if n == 0.0:
        if scale_ref is None:
            return 0.0 if d == 0.0 else float("inf")
        n = np.linalg.norm(np.asarray(scale_ref).ravel())
        if n == 0.0:
            return 0.0 if d == 0.0 else float("inf")
    return float(d / n)


def componentwise_err(C_hat: np.ndarray, C_ref: np.ndarray, absAB: np.ndarray) -> float:
    """max |C_hat - C_ref| / (|A|.|B|) over the entries where the bound is non-zero."""
    diff = np.abs(np.asarray(C_hat, dtype=np.float64) - C_ref)
    den = np.asarray(absAB, dtype=np.float64)
    mask = den > 0
    if np.any(diff[~mask] != 0):
        return float("inf")
    return float(np.max(diff[mask] / den[mask])) if np.any(mask) else 0.0


def gamma(k: int, u: float) -> float:
    """Higham's gamma_k = k u / (1 - k u), the classical bound on the relative
    error of a k-term dot product (Accuracy and Stability of Numerical
    Algorithms, 2nd ed., Section 3.1)."""
    return k * u / (1.0 - k * u)
