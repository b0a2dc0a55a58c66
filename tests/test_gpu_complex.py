"""GPU parity of complex contractions (TC_C128, TC_C64) against the complex
oracle, through the C ABI.  Tolerances: normwise 1e-12 (c128) and 1e-5 (c64,
against the oracle on the FP32-rounded parts); integer-valued parts bit-exact."""
import zlib

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_1409_8608_amd")


def _torch():
    import torch
    return torch


def tdtype(dtype):
    torch = _torch()
    return torch.complex128 if dtype == "c128" else torch.complex64


def crand(rng, shape, integer=False):
    if integer:
        x = rng.integers(-3, 4, size=shape) + 1j * rng.integers(-3, 4, size=shape)
    else:
        x = rng.uniform(-1, 1, size=shape) + 1j * rng.uniform(-1, 1, size=shape)
    return np.array(x, dtype=np.complex128, order="F")


def rounded(x, dtype):
    return x if dtype == "c128" else np.array(x.astype(np.complex64), dtype=np.complex128, order="F")


def device(x, dtype, strides=None):
    """Device copy of x, Fortran order or the given element strides."""
    torch = _torch()
    if strides is None:
        return tc.to_device_fortran(x, tdtype(dtype))
    span = 1 + sum((n - 1) * s for n, s in zip(x.shape, strides)) if x.size else 1
    store = torch.full((span,), complex(np.nan, np.nan), dtype=tdtype(dtype), device="cuda")
    t = torch.as_strided(store, tuple(x.shape), tuple(strides))
    t.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return t


def run(plan, A, B, C0, dtype, alpha=1.0, beta=0.0, strides=None):
    torch = _torch()
    strides = strides or {}
    dA, dB = device(A, dtype, strides.get("A")), device(B, dtype, strides.get("B"))
    if C0 is None:
        dC = device(np.full(plan.shape("C"), complex(np.nan, np.nan), order="F"), dtype, strides.get("C"))
    else:
        dC = device(C0, dtype, strides.get("C"))
    plan.contract(dA, dB, dC, complex(alpha), complex(beta))
    torch.cuda.synchronize()
    return dC.cpu().numpy().astype(np.complex128)


def check(spec, ext, A, B, got, dtype, C0=None, alpha=1.0, beta=0.0, exact=False):
    Ar, Br = rounded(A, dtype), rounded(B, dtype)
    Cr = None if C0 is None else rounded(C0, dtype)
    ref = oracle.contract(spec, ext, Ar, Br, C=Cr, alpha=alpha, beta=beta)
    if exact:
        np.testing.assert_array_equal(got, ref)
        return
    err = oracle.normwise_rel_err(got, ref)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert err <= tol, f"normwise error {err:.3e} > {tol:.1e}"


def operands(spec, ext, rng, integer=False, with_c=False):
    sa, sb, sc = oracle.split_spec(spec)
    A = crand(rng, [ext[ch] for ch in sa], integer)
    B = crand(rng, [ext[ch] for ch in sb], integer)
    C0 = crand(rng, [ext[ch] for ch in sc], integer) if with_c else None
    return A, B, C0


# Paths: streaming (few summed positions), matrix core with ragged tiles,
# permuted operands, batch and trace indices, an outer product (only the re/im
# index is summed), and B as the expanded (smaller) operand.
CASES = [
    ("abc=ai,ibc", dict(a=37, b=29, c=3, i=8)),
    ("abc=ai,ibc", dict(a=200, b=70, c=3, i=40)),
    ("abc=ija,jbic", dict(a=72, b=40, c=6, i=6, j=5)),
    ("ab=iaj,jbi", dict(a=130, b=90, i=7, j=9)),
    ("abcd=ai,ibcd", dict(a=50, b=6, c=5, d=4, i=12)),
    ("a=iaj,ji", dict(a=150, i=9, j=11)),
    ("abc=aic,ibc", dict(a=40, b=33, c=5, i=20)),
    ("ab=ai,ibt", dict(a=60, b=45, i=10, t=3)),
    ("ab=a,b", dict(a=70, b=50)),
    ("ab=ia,ib", dict(a=300, b=20, i=64)),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("spec,ext", CASES)
def test_complex_parity(spec, ext, dtype):
    rng = np.random.default_rng(zlib.crc32(repr((spec, sorted(ext.items()))).encode()))
    A, B, _ = operands(spec, ext, rng)
    p = tc.Plan(spec, ext, dtype)
    got = run(p, A, B, None, dtype)
    check(spec, ext, A, B, got, dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("spec,ext", CASES[:4] + CASES[6:])
def test_complex_integer_exact_with_alpha_beta(spec, ext, dtype):
    # small integer parts and alpha, beta in {+-1, +-i, 2}: every product and sum is
    # exact in either precision, so the result is unique whatever the order
    rng = np.random.default_rng(7)
    A, B, C0 = operands(spec, ext, rng, integer=True, with_c=True)
    p = tc.Plan(spec, ext, dtype)
    for alpha, beta in ((1.0, 0.0), (1j, -1.0), (-2.0, 1j), (1 + 1j, 1.0)):
        got = run(p, A, B, C0, dtype, alpha, beta)
        check(spec, ext, A, B, got, dtype, C0, alpha, beta, exact=True)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_complex_strided_operands(dtype):
    # padded leading dimensions in every operand, and C with permuted strides
    spec, ext = "abc=ai,ibc", dict(a=45, b=20, c=3, i=33)
    strides = dict(A=[1, 48], B=[1, 40, 40 * 21], C=[3 * 21, 3, 1])
    rng = np.random.default_rng(8)
    A, B, C0 = operands(spec, ext, rng, with_c=True)
    p = tc.Plan(spec, ext, dtype, strides=strides)
    got = run(p, A, B, C0, dtype, 0.5 - 0.25j, -1j, strides=strides)
    check(spec, ext, A, B, got, dtype, C0, 0.5 - 0.25j, -1j)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_complex_degenerate(dtype):
    torch = _torch()
    rng = np.random.default_rng(9)
    spec, ext = "ab=ai,ib", dict(a=9, b=7, i=5)
    A, B, C0 = operands(spec, ext, rng, integer=True, with_c=True)
    p = tc.Plan(spec, ext, dtype)
    # alpha == 0: A and B are not read (NaN there), C := beta C with complex beta
    nanA = np.full_like(A, complex(np.nan, np.nan))
    nanB = np.full_like(B, complex(np.nan, np.nan))
    got = run(p, nanA, nanB, C0, dtype, 0.0, 1 - 1j)
    np.testing.assert_array_equal(got, rounded(C0, dtype) * (1 - 1j))
    # beta == 0 with a NaN C: C is not read
    got = run(p, A, B, None, dtype, 1.0, 0.0)
    check(spec, ext, A, B, got, dtype, exact=True)
    # no summed positions: C := beta C
    ext0 = dict(ext, i=0)
    p0 = tc.Plan(spec, ext0, dtype)
    got = run(p0, np.zeros((9, 0), np.complex128, order="F"), np.zeros((0, 7), np.complex128, order="F"), C0, dtype,
              2.0, 1j)
    np.testing.assert_array_equal(got, rounded(C0, dtype) * 1j)
    # empty C: nothing to do
    pe = tc.Plan(spec, dict(ext, a=0), dtype)
    dC = torch.empty((0, 7), dtype=tdtype(dtype), device="cuda")
    pe.contract(device(np.zeros((0, 5), np.complex128, order="F"), dtype), device(B, dtype), dC, 1.0, 0.0)
    torch.cuda.synchronize()


def test_complex_fullsize_sampled():
    # 2048 x 2048 outputs, 512 summed positions (a matrix-core launch of
    # 4096 x 2048 real outputs and 1024 real positions); sampled rows and columns
    # against the oracle on the matching slices
    torch = _torch()
    spec, ext = "ab=ai,ib", dict(a=2048, b=2048, i=512)
    rng = np.random.default_rng(10)
    A, B, _ = operands(spec, ext, rng)
    p = tc.Plan(spec, ext, "c128")
    dA, dB = device(A, "c128"), device(B, "c128")
    dC = tc.empty_fortran([2048, 2048], torch.complex128)
    p.contract(dA, dB, dC, 1.0 + 0j, 0j)
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(2048, 24, replace=False))
    cols = np.sort(rng.choice(2048, 24, replace=False))
    got = dC.cpu().numpy()[np.ix_(rows, cols)]
    ref = oracle.contract(spec, dict(a=24, b=24, i=512), np.asfortranarray(A[rows]), np.asfortranarray(B[:, cols]))
    assert oracle.normwise_rel_err(got, ref) <= 1e-12


def test_complex_predict_and_workspace():
    torch = _torch()
    spec, ext = "abc=ai,ibc", dict(a=64, b=48, c=4, i=16)
    p = tc.Plan(spec, ext, "c128")
    pred = p.predict()
    assert len(pred) == 1 and pred[0]["variant"] == tc.TC_VARIANT_FUSED
    assert 0 < pred[0]["predicted_s"] < 1.0
    p.set_variant(tc.TC_VARIANT_PREDICTED)
    p.prepare()
    # the expanded operand (A, the smaller) takes four reals per complex element
    assert tc.tc_plan_workspace(p.handle) >= 4 * 64 * 16 * 8
    rng = np.random.default_rng(11)
    A, B, _ = operands(spec, ext, rng)
    got = run(p, A, B, None, "c128")
    check(spec, ext, A, B, got, "c128")
    # a second call on the same plan reuses the workspace
    A2, B2, _ = operands(spec, ext, rng)
    got = run(p, A2, B2, None, "c128")
    check(spec, ext, A2, B2, got, "c128")
    torch.cuda.synchronize()


# Complex streaming kernel: M a whole number of wave spans along C's unit
# stride (narrow lanes: 64 complex doubles, 128 complex floats; wide lanes:
# twice that), at most 8 summed positions (template sizes 4 and 8; the 12- and
# 16-position cases take the embedding), N not a multiple of the block's
# columns, two summed dims, C's unit stride in B (operands swapped), a trace
# index, an outer product, and padded operands (M = 128 takes the narrow form of
# complex floats, M = 256 the wide one).
ZSTREAM_CASES = [
    ("abc=ai,ibc", dict(a=128, b=20, c=3, i=8), None),
    ("abc=ai,ibc", dict(a=256, b=9, c=5, i=3), None),
    ("abc=ai,ibc", dict(a=128, b=7, c=3, i=16), None),
    ("ab=aij,jib", dict(a=256, b=30, i=3, j=4), None),
    ("ba=ai,ib", dict(a=20, b=128, i=6), None),
    ("ab=ai,ibt", dict(a=128, b=10, i=4, t=2), None),
    ("ab=a,b", dict(a=128, b=33), None),
    ("ab=ai,ib", dict(a=128, b=21, i=5), dict(A=[1, 128], B=[1, 5], C=[1, 130])),
    ("abc=ai,ibc", dict(a=512, b=11, c=2, i=7), None),
    ("ab=ai,ib", dict(a=256, b=9, i=6), dict(A=[1, 258], B=[1, 6], C=[1, 258])),
]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("spec,ext,strides", ZSTREAM_CASES)
def test_complex_streaming_parity(spec, ext, strides, dtype):
    rng = np.random.default_rng(zlib.crc32(repr((spec, sorted(ext.items()))).encode()))
    A, B, C0 = operands(spec, ext, rng, with_c=True)
    p = tc.Plan(spec, ext, dtype, strides=strides)
    got = run(p, A, B, None, dtype, strides=strides)
    check(spec, ext, A, B, got, dtype)
    got = run(p, A, B, C0, dtype, 0.5 + 2j, -0.75 + 0.5j, strides=strides)
    check(spec, ext, A, B, got, dtype, C0, 0.5 + 2j, -0.75 + 0.5j)
    Ai, Bi, Ci = operands(spec, ext, rng, integer=True, with_c=True)
    for alpha, beta in ((1.0, 0.0), (1j, 1 - 1j), (-2.0, 1.0)):
        got = run(p, Ai, Bi, Ci, dtype, alpha, beta, strides=strides)
        check(spec, ext, Ai, Bi, got, dtype, Ci, alpha, beta, exact=True)


@pytest.mark.parametrize("dtype,offset", [("c64", 1), ("c64", 2), ("c128", 1), ("c128", 0)])
def test_complex_streaming_alignment_forms(dtype, offset):
    # A starting `offset` complex elements into an allocation: a 16-byte-aligned
    # start keeps the streaming kernel (wide lane form at M = 256), an
    # 8-byte-aligned one takes the embedded real form
    torch = _torch()
    spec, ext = "abc=ai,ibc", dict(a=256, b=6, c=4, i=8)
    rng = np.random.default_rng(21)
    A, B, _ = operands(spec, ext, rng, integer=True)
    p = tc.Plan(spec, ext, dtype)
    store = torch.zeros(offset + 256 * 8, dtype=tdtype(dtype), device="cuda")
    dA = torch.as_strided(store, (256, 8), (1, 256), offset)
    dA.copy_(torch.from_numpy(A))
    dB = device(B, dtype)
    dC = tc.empty_fortran([256, 6, 4], tdtype(dtype))
    p.contract(dA, dB, dC, 1 + 0j, 0j)
    torch.cuda.synchronize()
    check(spec, ext, A, B, dC.cpu().numpy().astype(np.complex128), dtype, exact=True)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("compute,tol", [("bf16x3", 1e-5), ("fp8x3", 2e-3)])
@pytest.mark.parametrize("spec,ext", [("abc=ai,ibc", dict(a=96, b=40, c=3, i=40)),
                                      ("abc=ija,jbic", dict(a=72, b=40, c=6, i=6, j=5)),
                                      ("ab=ia,ib", dict(a=300, b=20, i=64))])
def test_complex_split_precision(spec, ext, dtype, compute, tol):
    """The split forms on the embedded real operands, against the complex oracle
    (normwise, as for real operands)."""
    rng = np.random.default_rng(31)
    A, B, C0 = operands(spec, ext, rng, with_c=True)
    p = tc.Plan(spec, ext, dtype, compute=compute)
    got = run(p, A, B, C0, dtype, 1 - 0.5j, 0.5j)
    ref = oracle.contract(spec, ext, rounded(A, dtype), rounded(B, dtype), C=rounded(C0, dtype), alpha=1 - 0.5j,
                          beta=0.5j)
    err = oracle.normwise_rel_err(got, ref)
    assert err <= tol, f"normwise error {err:.3e} > {tol:.1e}"
    rows, kp = tc.tc_split_terms(p.handle, 0, fp8=compute == "fp8x3")[0].shape[1:]
    assert rows > 0 and kp > 0
