"""Seeded synthetic inputs for the benchmark and test workloads.

Only random numbers and shapes live here -- none of the contraction
arithmetic -- so the GPU path and the CPU oracle can both take their inputs
from it.  Every array is float64 on the host in Fortran (column-major) order,
the paper's storage (Section 1); FP32 runs round these same values.

Workloads (the paper uses dense synthetic tensors defined by shape only):
  smallk_cube(n, i)   C_abc = A_ai B_ibc, a = b = c = n, contracted i
                      (Section 3 case study, i = 8); uniform[-1, 1];
                      seed 11 for n = 64, else 20 + n // 128
  permuted(...)       C_abc = A_ija B_jbic (Section 4.3 Test 3); normal(0, 1), seed 31
  scaled_matrix(...)  C_ab = A_iaj B_jbi with every free-index slice A[:, a, :]
                      and B[:, b, :] scaled by its own log-uniform[1e-3, 1e3]
                      factor; normal(0, 1), seed 41
  batch(...)          4096 contractions drawn from four patterns; seed 51
  complex_smallk(n, i), complex_square(m)
                      complex128 forms of smallk_cube (seed 61) and of a square
                      product C_ab = A_ai B_ib, a = b = i = m (seed 71); real and
                      imaginary parts uniform[-1, 1], drawn parts-first per operand
Draw order within one generator: A's entries, A's scales, B's entries, B's
scales, then C (only when an input C is requested).
"""
from __future__ import annotations

import numpy as np

PATTERNS = ("abc=ai,ibc", "abc=ija,jbic", "ab=iaj,jbi", "abcd=ai,ibcd")


def _split(spec):
    out, ins = spec.split("=")
    a, b = ins.split(",")
    return a, b, out


def _shape(letters, ext):
    return [int(ext[ch]) for ch in letters]


def tensors(spec: str, ext: dict, rng: np.random.Generator, dist: str = "uniform", with_c: bool = False,
            integer: bool = False):
    """A, B (and C) for `spec` drawn from `rng`; Fortran order, float64."""
    sa, sb, sc = _split(spec)

    def draw(letters):
        shape = _shape(letters, ext)
        if integer:
            x = rng.integers(-2, 3, size=shape).astype(np.float64)
        elif dist == "normal":
            x = rng.standard_normal(size=shape)
        else:
            x = rng.uniform(-1.0, 1.0, size=shape)
        return np.array(x, order="F")

    A = draw(sa)
    B = draw(sb)
    C = draw(sc) if with_c else None
    return A, B, C


def smallk_cube(n: int = 64, i: int = 8, integer: bool = False, with_c: bool = False):
    spec = "abc=ai,ibc"
    ext = dict(a=n, b=n, c=n, i=i)
    seed = 11 if n == 64 else 20 + n // 128
    A, B, C = tensors(spec, ext, np.random.default_rng(seed), "uniform", with_c, integer)
    return dict(spec=spec, ext=ext, A=A, B=B, C=C, seed=seed)


def permuted(n: int = 256, k: int = 32, integer: bool = False, with_c: bool = False, seed: int = 31):
    spec = "abc=ija,jbic"
    ext = dict(a=n, b=n, c=n, i=k, j=k)
    A, B, C = tensors(spec, ext, np.random.default_rng(seed), "normal", with_c, integer)
    return dict(spec=spec, ext=ext, A=A, B=B, C=C, seed=seed)


def scaled_matrix(n: int = 4096, k: int = 64, seed: int = 41):
    """C_ab = A_iaj B_jbi; slice A[:, a, :] times s_a, B[:, b, :] times s_b,
    s log-uniform on [1e-3, 1e3]."""
    spec = "ab=iaj,jbi"
    ext = dict(a=n, b=n, i=k, j=k)
    rng = np.random.default_rng(seed)
    lo, hi = np.log(1e-3), np.log(1e3)
    A = np.array(rng.standard_normal(size=(k, n, k)), order="F")
    sA = np.exp(rng.uniform(lo, hi, size=n))
    A *= sA[None, :, None]
    B = np.array(rng.standard_normal(size=(k, n, k)), order="F")
    sB = np.exp(rng.uniform(lo, hi, size=n))
    B *= sB[None, :, None]
    return dict(spec=spec, ext=ext, A=A, B=B, C=None, seed=seed, scales=(sA, sB))


def _logu_int(rng, lo, hi):
    return int(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi)))))


def batch_shapes(count: int = 4096, seed: int = 51, cap_elems: int = 1 << 24, free=(8, 256), con=(4, 64)):
    """Patterns uniform over PATTERNS; free extents log-uniform integers in
    `free` ([8, 256]), contracted extents in `con` ([4, 64]); a draw whose
    largest operand exceeds `cap_elems` elements is drawn again from the same
    stream."""
    rng = np.random.default_rng(seed)
    con_rng = con
    out = []
    redraws = 0
    while len(out) < count:
        spec = PATTERNS[int(rng.integers(0, len(PATTERNS)))]
        sa, sb, sc = _split(spec)
        con_idx = [ch for ch in sa if ch in sb]
        ext = {}
        for ch in sorted(set(sa + sb + sc)):
            ext[ch] = _logu_int(rng, *con_rng) if ch in con_idx else _logu_int(rng, *free)
        biggest = max(int(np.prod(_shape(x, ext))) for x in (sa, sb, sc))
        if biggest > cap_elems:
            redraws += 1
            continue
        out.append(dict(spec=spec, ext=ext))
    children = np.random.SeedSequence(seed).spawn(count)
    for item, ss in zip(out, children):
        item["seed_seq"] = ss
    return out, redraws


def batch_values(item: dict, integer: bool = False):
    """A, B of one batch member, uniform[-1, 1], from its own spawned seed."""
    rng = np.random.default_rng(item["seed_seq"])
    A, B, _ = tensors(item["spec"], item["ext"], rng, "uniform", False, integer)
    return A, B


def complex_tensors(spec: str, ext: dict, rng: np.random.Generator):
    """Complex A and B for `spec`: real part then imaginary part of A, then of B,
    each uniform[-1, 1]; Fortran order, complex128."""
    sa, sb, _ = _split(spec)

    def draw(letters):
        shape = _shape(letters, ext)
        re = rng.uniform(-1.0, 1.0, size=shape)
        im = rng.uniform(-1.0, 1.0, size=shape)
        return np.array(re + 1j * im, dtype=np.complex128, order="F")

    A = draw(sa)
    B = draw(sb)
    return A, B


def complex_smallk(n: int = 1024, i: int = 8):
    spec = "abc=ai,ibc"
    ext = dict(a=n, b=n, c=n, i=i)
    A, B = complex_tensors(spec, ext, np.random.default_rng(61))
    return dict(spec=spec, ext=ext, A=A, B=B)


def complex_square(m: int = 4096):
    spec = "ab=ai,ib"
    ext = dict(a=m, b=m, i=m)
    A, B = complex_tensors(spec, ext, np.random.default_rng(71))
    return dict(spec=spec, ext=ext, A=A, B=B)
