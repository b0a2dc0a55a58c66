"""Helpers shared by the GPU tests: move seeded host inputs to the device in
the plan's layout, run the library, bring C back, compare with the oracle."""
from __future__ import annotations

import numpy as np

import oracle


def torch_mod():
    import torch
    return torch


def run(plan, A, B, C0=None, alpha=1.0, beta=0.0, dtype="f64"):
    """Run ``plan`` on host arrays (Fortran order) and return C as float64."""
    import paper_1409_8608_amd as tc
    torch = torch_mod()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    dA = tc.to_device_fortran(A, tdt)
    dB = tc.to_device_fortran(B, tdt)
    if C0 is not None:
        dC = tc.to_device_fortran(C0, tdt)
    else:
        dC = tc.empty_fortran(plan.shape("C"), tdt)
        dC.fill_(float("nan"))             # beta = 0 must not read C
    plan.contract(dA, dB, dC, alpha, beta)
    torch.cuda.synchronize()
    out = dC.double().cpu().numpy()
    return out


def rounded(x, dtype):
    """Values the device actually sees (FP32 runs round the FP64 draws)."""
    return x if dtype == "f64" else x.astype(np.float32).astype(np.float64)


def check(spec, ext, A, B, got, dtype="f64", C0=None, alpha=1.0, beta=0.0, exact=False, tol=None):
    # np.array(..., order="F") keeps 0-d operands arrays (ufuncs return scalars)
    Ar, Br = np.array(rounded(A, dtype), order="F"), np.array(rounded(B, dtype), order="F")
    Cr = None if C0 is None else np.array(rounded(C0, dtype), order="F")
    ref = oracle.contract(spec, ext, Ar, Br, C=Cr, alpha=alpha, beta=beta)
    if exact:
        np.testing.assert_array_equal(got, ref)
        return 0.0
    absAB = oracle.contract(spec, ext, np.array(np.abs(Ar), order="F"), np.array(np.abs(Br), order="F"))
    err = oracle.normwise_rel_err(got, ref, absAB)
    if tol is None:
        tol = 1e-12 if dtype == "f64" else 1e-5
    assert err <= tol, f"normwise error {err:.3e} > {tol:.1e}"
    return err


def split_bound(K: int, small: int = 5) -> float:
    """Componentwise bound, relative to (|A||B|)_c, between the device's
    split-BF16 result and the oracle's exactly accumulated split result.
    The leading product t_A1 t_B1 accumulates in FP32 over all K positions:
    (K + 8) u with u = 2^-24, each product rounded into the sum in the worst
    case.  The `small` other products (five by default; each at most about
    2^-7 of the leading one per position) accumulate in a second FP32 sum:
    small K u 2^-7.  2^-22 covers the FP64 combine and the unscaling."""
    return (K + 8) * 2.0 ** -24 + small * K * 2.0 ** -31 + 2.0 ** -22


def split_bound_fp8(K: int) -> float:
    """split_bound for OCP E4M3 terms.  The small products are together at
    most 2^-3 of the leading one per position (each term carries 4 significant
    bits), so their FP32 sum contributes 5 K u 2^-3.  The FP8 matrix
    instructions of MI355X add their products with less than FP32 precision:
    measured on one instruction with random normal-range E4M3 operands, up to
    880 u of the instruction's sum of |products| (about 2^-14), against about
    1 u for the BF16 instructions; 2^-12 |A||B| covers it."""
    return (K + 8) * 2.0 ** -24 + 5 * K * 2.0 ** -27 + 2.0 ** -12


def e4m3_value(codes):
    """Values of OCP E4M3 codes (uint8 array)."""
    import numpy as np
    c = np.asarray(codes).astype(np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 15
    m = (c & 7).astype(np.float64)
    v = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    return s * v
