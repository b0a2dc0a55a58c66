"""Pins for the split-precision oracle: the rounding routines against their
definitions (nearest representable value by exhaustive neighbourhood search,
ties to even, exactly representable values fixed), the split identities, the
error of the three-term form against the exact contraction, and exactness on
small integers."""
import numpy as np
import pytest

import oracle
from oracle import split as sp


def _bf16_grid(E):
    """All 8-bit-significand values with leading exponent E (|x| in [2^E, 2^(E+1)))."""
    s = np.arange(128, 256, dtype=np.float64)
    return np.ldexp(s, E - 7)


def test_round_bits_is_nearest_even():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))
    r = sp.round_bits(x, 8)
    for xi, ri in zip(x[:3000], r[:3000]):
        E = int(np.floor(np.log2(abs(xi))))
        cand = np.concatenate([_bf16_grid(E - 1), _bf16_grid(E), _bf16_grid(E + 1)]) * np.sign(xi)
        d = np.abs(cand - xi)
        best = cand[d == d.min()]
        assert ri in best
        if len(best) == 2:    # a tie: the even significand wins
            sig = [int(abs(b) / 2.0 ** (np.floor(np.log2(abs(b))) - 7)) for b in best]
            assert int(abs(ri) / 2.0 ** (np.floor(np.log2(abs(ri))) - 7)) % 2 == 0
    assert np.all(np.abs(r - x) <= np.ldexp(np.abs(x), -8))     # half an ulp of an 8-bit significand


def test_round_bits_ties_and_exact_values():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: the even neighbour is 1
    assert sp.round_bits(np.array([1 + 2.0 ** -8]), 8)[0] == 1.0
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert sp.round_bits(np.array([1 + 3 * 2.0 ** -8]), 8)[0] == 1 + 2.0 ** -6
    v = _bf16_grid(3)
    np.testing.assert_array_equal(sp.round_bits(v, 8), v)
    np.testing.assert_array_equal(sp.round_bits(-v, 8), -v)
    assert sp.round_bits(np.array([0.0]), 8)[0] == 0.0


def test_round_e4m3():
    # normal values with 4 significant bits stay, 448 is the largest, subnormal spacing 2^-9
    vals = np.array([1.0, 1.125, 1.875, 448.0, 2.0 ** -6, 2.0 ** -9, 3 * 2.0 ** -9, -240.0])
    np.testing.assert_array_equal(sp.round_e4m3(vals), vals)
    assert sp.round_e4m3(np.array([1.0625]))[0] == 1.0          # tie -> even
    assert sp.round_e4m3(np.array([1.1875]))[0] == 1.25         # tie -> even
    assert sp.round_e4m3(np.array([1000.0]))[0] == 448.0        # saturates
    assert sp.round_e4m3(np.array([2.0 ** -11]))[0] == 0.0      # below half the smallest subnormal


def test_split_identities_and_error():
    rng = np.random.default_rng(1)
    X = np.array(rng.standard_normal((16, 40)) * np.exp(rng.uniform(-5, 5, (1, 40))), order="F")
    T, e = sp.split_terms(X, "ka", "a")
    xs = np.ldexp(X, -e[None, :])
    assert np.all(np.max(np.abs(xs), axis=0) >= 1.0) and np.all(np.max(np.abs(xs), axis=0) < 2.0)
    # every term is an 8-bit value, t1 + r1 = xs exactly, and the residual after three terms is tiny
    for t in T:
        np.testing.assert_array_equal(sp.round_bits(t, 8), t)
    assert np.all(np.abs(xs - (T[0] + T[1] + T[2])) <= np.ldexp(np.abs(xs), -24))
    # float32 inputs split exactly into three terms
    X32 = X.astype(np.float32).astype(np.float64)
    T32, e32 = sp.split_terms(X32, "ka", "a")
    np.testing.assert_array_equal(T32[0] + T32[1] + T32[2], np.ldexp(X32, -e32[None, :]))


def test_split_contraction_error_bound():
    """Dropping the products with p + q > 4 and the residual of the third term
    leaves an error far below FP32 level (about 2^-24 of |A||B|)."""
    rng = np.random.default_rng(2)
    spec, ext = "ab=iaj,jbi", dict(a=20, b=24, i=6, j=7)
    A = np.array(rng.standard_normal((6, 20, 7)) * np.exp(rng.uniform(-7, 7, (1, 20, 1))), order="F")
    B = np.array(rng.standard_normal((7, 24, 6)) * np.exp(rng.uniform(-7, 7, (1, 24, 1))), order="F")
    ref = oracle.contract(spec, ext, A, B)
    absAB = oracle.contract(spec, ext, np.abs(A), np.abs(B))
    got = sp.contract_split(spec, ext, A, B)
    assert np.all(np.abs(got - ref) <= 2.0 ** -22 * absAB)
    # with all nine products the error only shrinks
    got9 = sp.contract_split(spec, ext, A, B, pairs=[(p, q) for p in (1, 2, 3) for q in (1, 2, 3)])
    assert np.max(np.abs(got9 - ref) / absAB) <= np.max(np.abs(got - ref) / absAB) * 1.01 + 1e-300
    # one-term products are BF16-level only
    got1 = sp.contract_split(spec, ext, A, B, pairs=[(1, 1)])
    assert np.max(np.abs(got1 - ref) / absAB) > 1e-4


def test_split_product_ablations():
    """The term-product ablations of the split form.  With all nine products
    the split of FP32-representable operands is exact (three 8-bit terms hold
    24 bits), so the result is the plain contraction up to FP64 rounding.
    Keeping only p + q <= 3 drops t1 t3, t3 t1 and t2 t2, each at most about
    2^-16 of |a||b| (|t2| <= 2^-8 |x|, |t3| <= 2^-16 |x| after rounding to
    nearest), so the error is below 2^-14 |A||B|, and for random data far
    above the six-product error."""
    rng = np.random.default_rng(12)
    spec, ext = "ab=iaj,jbi", dict(a=18, b=21, i=5, j=9)
    A = np.array(rng.standard_normal((5, 18, 9)) * np.exp(rng.uniform(-6, 6, (1, 18, 1))), order="F")
    B = np.array(rng.standard_normal((9, 21, 5)) * np.exp(rng.uniform(-6, 6, (1, 21, 1))), order="F")
    A32, B32 = (x.astype(np.float32).astype(np.float64) for x in (A, B))
    all9 = [(p, q) for p in (1, 2, 3) for q in (1, 2, 3)]
    p3 = [(p, q) for p in (1, 2) for q in (1, 2) if p + q <= 3]
    assert sorted(p3) == [(1, 1), (1, 2), (2, 1)] and len(sp.PAIRS) == 6
    ref32 = oracle.contract(spec, ext, A32, B32)
    abs32 = oracle.contract(spec, ext, np.abs(A32), np.abs(B32))
    got9 = sp.contract_split(spec, ext, A32, B32, pairs=all9)
    assert np.all(np.abs(got9 - ref32) <= 2.0 ** -50 * abs32)
    ref = oracle.contract(spec, ext, A, B)
    absAB = oracle.contract(spec, ext, np.abs(A), np.abs(B))
    e3 = np.max(np.abs(sp.contract_split(spec, ext, A, B, pairs=p3) - ref) / absAB)
    e6 = np.max(np.abs(sp.contract_split(spec, ext, A, B) - ref) / absAB)
    assert e3 <= 2.0 ** -14 and e3 > 2.0 ** -20 and e6 < 2.0 ** -22


def test_split_integer_exact():
    """Small integers are exact in one BF16 (or E4M3) term: the split form
    equals the plain contraction bit for bit."""
    rng = np.random.default_rng(3)
    spec, ext = "abc=ija,jbic", dict(a=5, b=4, c=3, i=6, j=2)
    A = np.array(rng.integers(-3, 4, (6, 2, 5)).astype(float), order="F")
    B = np.array(rng.integers(-3, 4, (2, 4, 6, 3)).astype(float), order="F")
    ref = oracle.contract(spec, ext, A, B)
    for kind in ("bf16", "fp8"):
        np.testing.assert_array_equal(sp.contract_split(spec, ext, A, B, kind=kind), ref)


def test_fp8_split_error():
    rng = np.random.default_rng(4)
    spec, ext = "ab=ai,ib", dict(a=30, b=20, i=50)
    A = np.array(rng.standard_normal((30, 50)), order="F")
    B = np.array(rng.standard_normal((50, 20)), order="F")
    ref = oracle.contract(spec, ext, A, B)
    absAB = oracle.contract(spec, ext, np.abs(A), np.abs(B))
    got = sp.contract_split(spec, ext, A, B, kind="fp8")
    err = np.max(np.abs(got - ref) / absAB)
    assert err < 2.0 ** -9            # three 4-bit terms: about 12 significant bits
    assert err > 2.0 ** -30           # and clearly not exact


def test_slice_exponents_permuted_free_axes():
    """Free axes in a different order in the operand and in C."""
    rng = np.random.default_rng(5)
    spec, ext = "ab=bia,i", dict(a=3, b=4, i=5)
    A = np.array(rng.standard_normal((4, 5, 3)) * np.exp(rng.uniform(-9, 9, (4, 1, 3))), order="F")
    B = np.array(rng.standard_normal(5), order="F")
    ref = oracle.contract(spec, ext, A, B)
    absAB = oracle.contract(spec, ext, np.abs(A), np.abs(B))
    got = sp.contract_split(spec, ext, A, B)
    assert np.all(np.abs(got - ref) <= 2.0 ** -22 * absAB)
