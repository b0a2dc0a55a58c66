"""GPU parity of the split-BF16 precision form against its oracle (the same
steps with exact accumulation) and against the plain FP64 contraction."""
import numpy as np
import pytest

import oracle
from oracle import split as sp
from gpu_util import e4m3_value, run, split_bound, split_bound_fp8

pytestmark = pytest.mark.gpu
tc = pytest.importorskip("paper_1409_8608_amd")
from paper_1409_8608_amd import workloads as wl  # noqa: E402


def _bf16_value(bits):
    """BF16 bit patterns -> float64 values (upper half of an FP32 pattern)."""
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_integer_exact(dtype):
    """Small integers are single BF16 terms and every FP32 partial sum is exact:
    the split form must equal the plain contraction bit for bit."""
    spec, ext = "abc=ija,jbic", dict(a=70, b=20, c=9, i=13, j=17)
    A, B, C = wl.tensors(spec, ext, np.random.default_rng(5), integer=True, with_c=True)
    p = tc.Plan(spec, ext, dtype, compute="bf16x3")
    got = run(p, A, B, C, alpha=1.0, beta=2.0, dtype=dtype)
    np.testing.assert_array_equal(got, oracle.contract(spec, ext, A, B, C=np.array(C, order="F"), alpha=1.0, beta=2.0))


@pytest.mark.parametrize("spec,ext", [
    ("ab=iaj,jbi", dict(a=130, b=200, i=24, j=17)),
    ("abc=ija,jbic", dict(a=40, b=33, c=7, i=5, j=11)),
    ("abcd=ai,ibcd", dict(a=17, b=5, c=6, d=7, i=300)),
])
def test_split_terms_bit_exact_and_result(spec, ext):
    """The device's exponents and BF16 terms equal the oracle's bit for bit,
    and the result is within the FP32-accumulation bound of the oracle's
    exactly accumulated split result, and at FP32 level against FP64."""
    rng = np.random.default_rng(9)
    sa, sb, sc = oracle.split_spec(spec)
    A = np.array(rng.standard_normal([ext[c] for c in sa]), order="F")
    B = np.array(rng.standard_normal([ext[c] for c in sb]), order="F")
    # per-slice scales over several binades (free-index slices)
    fa = [ax for ax, ch in enumerate(sa) if ch in sc]
    A *= np.exp(rng.uniform(np.log(1e-3), np.log(1e3), [A.shape[ax] if ax in fa else 1 for ax in range(A.ndim)]))
    p = tc.Plan(spec, ext, "f64", compute="bf16x3")
    got = run(p, A, B)
    ref_split = sp.contract_split(spec, ext, A, B)
    ref = oracle.contract(spec, ext, A, B)
    absAB = oracle.contract(spec, ext, np.abs(A), np.abs(B))
    K = int(np.prod([ext[c] for c in sa if c not in sc]))
    bound = split_bound(K)
    assert np.all(np.abs(got - ref_split) <= bound * absAB)
    assert oracle.normwise_rel_err(got, ref) <= 1e-5
    # exponents: one per free multi-index, first free index fastest (the GEMM view's rows)
    tA, eA = tc.tc_split_terms(p.handle, 0)
    want_e = sp.slice_exponents(A, sa, "".join(c for c in sa if c in sc))
    np.testing.assert_array_equal(eA, np.asarray(want_e).ravel(order="F"))
    # terms: the multiset of values per row must equal the oracle's (the device packs in its K order)
    TA, _ = sp.split_terms(A, sa, "".join(c for c in sa if c in sc))
    free_axes = [ax for ax, ch in enumerate(sa) if ch in sc]
    con_axes = [ax for ax, ch in enumerate(sa) if ch not in sc]
    for t in range(3):
        dev = _bf16_value(tA[t])                              # rows x kp (K order + zero padding)
        ora = np.transpose(TA[t], free_axes + con_axes).reshape(len(eA), -1, order="F") \
            if len(free_axes) == 1 else None
        if ora is None:
            continue
        for r in range(0, len(eA), max(1, len(eA) // 16)):
            d = np.sort(dev[r][dev[r] != 0])
            o = np.sort(ora[r][ora[r] != 0])
            np.testing.assert_array_equal(d, o)


@pytest.mark.parametrize("products", [3, 9])
@pytest.mark.parametrize("spec,ext", [
    ("ab=iaj,jbi", dict(a=300, b=140, i=24, j=17)),
    ("abc=ija,jbic", dict(a=40, b=33, c=7, i=5, j=11)),
])
def test_split_product_ablations(spec, ext, products):
    """The ablations of the split-BF16 form: three term products (p + q <= 3)
    and all nine.  Componentwise within the FP32-accumulation bound of the
    oracle's exactly accumulated split result with the same products; the
    three-product form is BF16x2 level (about 2^-16 |A||B|), the nine-product
    form at least as accurate as the six-product one.  Batches refuse them."""
    rng = np.random.default_rng(19)
    sa, sb, sc = oracle.split_spec(spec)
    A = np.array(rng.standard_normal([ext[c] for c in sa]), order="F")
    B = np.array(rng.standard_normal([ext[c] for c in sb]), order="F")
    fa = [ax for ax, ch in enumerate(sa) if ch in sc]
    A *= np.exp(rng.uniform(np.log(1e-3), np.log(1e3), [A.shape[ax] if ax in fa else 1 for ax in range(A.ndim)]))
    pairs = [(p, q) for p in (1, 2, 3) for q in (1, 2, 3) if products == 9 or p + q <= 3]
    p = tc.Plan(spec, ext, "f64", compute="bf16x3", products=products)
    got = run(p, A, B)
    ref_split = sp.contract_split(spec, ext, A, B, pairs=pairs)
    ref = oracle.contract(spec, ext, A, B)
    absAB = oracle.contract(spec, ext, np.abs(A), np.abs(B))
    K = int(np.prod([ext[c] for c in sa if c not in sc]))
    assert np.all(np.abs(got - ref_split) <= split_bound(K, small=len(pairs) - 1) * absAB)
    err = np.max(np.abs(got - ref) / absAB)
    if products == 3:
        assert 2.0 ** -22 < err <= 2.0 ** -14
    else:
        p6 = tc.Plan(spec, ext, "f64", compute="bf16x3")
        err6 = np.max(np.abs(run(p6, A, B) - ref) / absAB)
        assert err <= err6 * 1.05 + 2.0 ** -40
        assert oracle.normwise_rel_err(got, ref) <= 1e-5
    with pytest.raises(tc.TcError) as e:
        tc.Batch([p])
    assert e.value.name == "TC_E_UNSUPPORTED"


def test_split_products_errors():
    with pytest.raises(tc.TcError) as e:
        tc.Plan("ab=ai,ib", dict(a=8, b=8, i=8), "f64", compute="bf16x3", products=4)
    assert e.value.name == "TC_E_UNSUPPORTED"
    with pytest.raises(tc.TcError) as e:
        tc.Plan("ab=ai,ib", dict(a=8, b=8, i=8), "f64", compute="fp8x3", products=3)
    assert e.value.name == "TC_E_UNSUPPORTED"


@pytest.mark.parametrize("K", [6000, 9000])
def test_split_long_contraction(K):
    """Long contracted extents: 4096 < K <= 8192 keeps each slice in
    registers (four chunks per thread); K > 8192 takes the two-pass form.
    Per-slice scales over six decades; the device's exponents equal the
    oracle's, and the result is within the FP32-accumulation bound of the
    exactly accumulated split oracle."""
    spec, ext = "ab=ai,ib", dict(a=40, b=70, i=K)
    rng = np.random.default_rng(K)
    A = np.array(rng.standard_normal((40, K)) * np.exp(rng.uniform(np.log(1e-3), np.log(1e3), (40, 1))), order="F")
    B = np.array(rng.standard_normal((K, 70)), order="F")
    p = tc.Plan(spec, ext, "f64", compute="bf16x3")
    got = run(p, A, B)
    ref_split = sp.contract_split(spec, ext, A, B)
    absAB = oracle.contract(spec, ext, np.abs(A), np.abs(B))
    assert np.all(np.abs(got - ref_split) <= split_bound(K) * absAB)
    assert oracle.normwise_rel_err(got, oracle.contract(spec, ext, A, B)) <= 1e-5
    _, eA = tc.tc_split_terms(p.handle, 0)
    np.testing.assert_array_equal(eA, np.asarray(sp.slice_exponents(A, "ai", "a")).ravel(order="F"))


@pytest.mark.parametrize("spec,ext", [
    ("ab=iaj,jbi", dict(a=130, b=200, i=24, j=17)),
    ("abc=ija,jbic", dict(a=40, b=33, c=7, i=5, j=11)),
    ("ab=ai,ib", dict(a=300, b=140, i=700)),
])
def test_fp8_terms_bit_exact_and_result(spec, ext):
    """FP8 (OCP E4M3) split: exponents equal the oracle's; each row's terms,
    decoded and unscaled, equal the oracle's as a multiset; the result is
    within the FP32-accumulation bound of the exactly accumulated FP8 split
    oracle and within the FP8 split's own 2^-9 of the FP64 contraction."""
    rng = np.random.default_rng(12)
    sa, sb, sc = oracle.split_spec(spec)
    A = np.array(rng.standard_normal([ext[c] for c in sa]), order="F")
    B = np.array(rng.standard_normal([ext[c] for c in sb]), order="F")
    fa = [ax for ax, ch in enumerate(sa) if ch in sc]
    A *= np.exp(rng.uniform(np.log(1e-3), np.log(1e3), [A.shape[ax] if ax in fa else 1 for ax in range(A.ndim)]))
    p = tc.Plan(spec, ext, "f64", compute="fp8x3")
    got = run(p, A, B)
    ref_split = sp.contract_split(spec, ext, A, B, kind="fp8")
    absAB = oracle.contract(spec, ext, np.abs(A), np.abs(B))
    K = int(np.prod([ext[c] for c in sa if c not in sc]))
    assert np.all(np.abs(got - ref_split) <= split_bound_fp8(K) * absAB)
    assert np.all(np.abs(got - oracle.contract(spec, ext, A, B)) <= 2.0 ** -9 * absAB)
    tA, eA = tc.tc_split_terms(p.handle, 0, fp8=True)
    free = "".join(c for c in sa if c in sc)
    np.testing.assert_array_equal(eA, np.asarray(sp.slice_exponents(A, sa, free)).ravel(order="F"))
    TA, _ = sp.split_terms(A, sa, free, kind="fp8")
    con_axes = [ax for ax, ch in enumerate(sa) if ch not in sc]
    if len(fa) == 1:
        for t in range(3):
            dev = e4m3_value(tA[t]) * 2.0 ** (-4 * t)
            ora = np.transpose(TA[t], fa + con_axes).reshape(len(eA), -1, order="F")
            for r in range(0, len(eA), max(1, len(eA) // 16)):
                np.testing.assert_array_equal(np.sort(dev[r][dev[r] != 0]), np.sort(ora[r][ora[r] != 0]))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scaled_matrix_accuracy(dtype):
    """The precision workload's shape at reduced size: slices scaled over six
    decades; FP32-level error against the FP64 contraction."""
    w = wl.scaled_matrix(n=256, k=16)
    p = tc.Plan(w["spec"], w["ext"], dtype, compute="bf16x3")
    got = run(p, w["A"], w["B"], dtype=dtype)
    Ar = w["A"] if dtype == "f64" else w["A"].astype(np.float32).astype(np.float64)
    Br = w["B"] if dtype == "f64" else w["B"].astype(np.float32).astype(np.float64)
    ref = oracle.contract(w["spec"], w["ext"], Ar, Br)
    err = oracle.normwise_rel_err(got, ref)
    assert err <= 1e-5, err


def test_split_rejects_members():
    p = tc.Plan("ab=ai,ib", dict(a=8, b=8, i=8), "f64", compute="bf16x3")
    with pytest.raises(tc.TcError) as e:
        p.set_variant(0)
    assert e.value.name == "TC_E_UNSUPPORTED"
