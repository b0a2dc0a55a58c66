"""Pins for the complex form of the oracle (the Section 1 sum over complex
numbers) against things other than itself: integer-valued complex inputs where
every rounding is exact (brute force with Python's complex type), numpy's
einsum, a product worked out by hand, the Gram matrix A A^H (Hermitian, real
diagonal equal to squared row norms), reduction to the real oracle for real
inputs, and complex alpha/beta."""
import itertools

import numpy as np
import pytest

import oracle

SPECS = ["abc=ai,ibc", "abc=ija,jbic", "ab=iaj,jbi", "abcd=ai,ibcd", "a=iaj,ji", "abc=aic,ibc", "ab=ai,ibt",
         "ab=a,b"]


def letters_of(spec):
    return sorted(set(spec.replace("=", "").replace(",", "")))


def crand(rng, letters, ext, integer=False):
    shape = [ext[ch] for ch in letters]
    if integer:
        x = rng.integers(-3, 4, size=shape) + 1j * rng.integers(-3, 4, size=shape)
    else:
        x = rng.uniform(-1, 1, size=shape) + 1j * rng.uniform(-1, 1, size=shape)
    return np.array(x, dtype=np.complex128, order="F")


def brute(spec, ext, A, B):
    """C[f] += A[.] B[.] over every assignment of every index, in Python complex."""
    sa, sb, sc = oracle.split_spec(spec)
    letters = letters_of(spec)
    C = np.zeros([ext[ch] for ch in sc], dtype=np.complex128)
    for vals in itertools.product(*[range(ext[ch]) for ch in letters]):
        v = dict(zip(letters, vals))
        a = complex(A[tuple(v[ch] for ch in sa)])
        b = complex(B[tuple(v[ch] for ch in sb)])
        C[tuple(v[ch] for ch in sc)] += a * b
    return C


@pytest.mark.parametrize("spec", SPECS)
def test_integer_complex_exact_vs_brute(spec):
    # small integer parts: every product and sum is exact in FP64, so the
    # result is unique whatever the order
    rng = np.random.default_rng(11)
    sa, sb, sc = oracle.split_spec(spec)
    ext = {ch: 2 + (q % 2) for q, ch in enumerate(letters_of(spec))}
    A, B = crand(rng, sa, ext, True), crand(rng, sb, ext, True)
    np.testing.assert_array_equal(oracle.contract(spec, ext, A, B), brute(spec, ext, A, B))


@pytest.mark.parametrize("spec", SPECS)
def test_matches_einsum(spec):
    rng = np.random.default_rng(12)
    sa, sb, sc = oracle.split_spec(spec)
    ext = {ch: 3 + (q % 3) for q, ch in enumerate(letters_of(spec))}
    A, B = crand(rng, sa, ext), crand(rng, sb, ext)
    got = oracle.contract(spec, ext, A, B)
    ref = np.einsum(f"{sa},{sb}->{sc}", A, B)
    assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


def test_hand_worked_product():
    # (1+2i)(3-i) = 5+5i and (i)(i) = -1 and 2(1+i) = 2+2i, (1-i)(2+i) = 3-i
    A = np.array([[1 + 2j, 1j], [2, 1 - 1j]], dtype=np.complex128, order="F")
    B = np.array([[3 - 1j, 1], [1j, 2 + 1j]], dtype=np.complex128, order="F")
    C = oracle.contract("ab=ai,ib", dict(a=2, b=2, i=2), A, B)
    # row 0: (1+2i)(3-i) + i*i = 4+5i ; (1+2i)*1 + i(2+i) = 1+2i+2i-1 = 4i
    # row 1: 2(3-i) + (1-i)i = 6-2i+i+1 = 7-i ; 2*1 + (1-i)(2+i) = 2+3-i = 5-i
    np.testing.assert_array_equal(C, np.array([[4 + 5j, 4j], [7 - 1j, 5 - 1j]]))


def test_gram_matrix_is_hermitian_with_row_norms():
    rng = np.random.default_rng(13)
    A = crand(rng, "ak", dict(a=6, k=9))
    AH = np.asfortranarray(A.conj().T)
    G = oracle.contract("ab=ak,kb", dict(a=6, b=6, k=9), A, AH)
    np.testing.assert_allclose(G, G.conj().T, rtol=0, atol=1e-14)
    assert np.all(G.diagonal().imag == 0.0)       # x conj(x) has an exactly zero imaginary part
    np.testing.assert_allclose(G.diagonal().real, (np.abs(A) ** 2).sum(axis=1), rtol=1e-14)


@pytest.mark.parametrize("spec", SPECS)
def test_real_inputs_reduce_to_real_oracle(spec):
    rng = np.random.default_rng(14)
    sa, sb, sc = oracle.split_spec(spec)
    ext = {ch: 2 + (q % 3) for q, ch in enumerate(letters_of(spec))}
    Ar, Br = crand(rng, sa, ext).real.copy(order="F"), crand(rng, sb, ext).real.copy(order="F")
    Cr = crand(rng, sc, ext).real.copy(order="F")
    real = oracle.contract(spec, ext, Ar, Br, C=Cr.copy(order="F"), alpha=0.75, beta=-1.5)
    cplx = oracle.contract(spec, ext, np.array(Ar, dtype=np.complex128, order="F"),
                           np.array(Br, dtype=np.complex128, order="F"),
                           C=np.array(Cr, dtype=np.complex128, order="F"), alpha=0.75, beta=-1.5)
    np.testing.assert_array_equal(cplx.real, real)
    assert np.all(cplx.imag == 0.0)


def test_four_real_contractions():
    # (Ar + i Ai)(Br + i Bi) = (Ar Br - Ai Bi) + i (Ar Bi + Ai Br), each a real
    # contraction of the already pinned real oracle
    rng = np.random.default_rng(15)
    spec, ext = "abc=ija,jbic", dict(a=3, b=4, c=2, i=3, j=2)
    sa, sb, sc = oracle.split_spec(spec)
    A, B = crand(rng, sa, ext), crand(rng, sb, ext)
    f = lambda x, y: oracle.contract(spec, ext, np.asfortranarray(x), np.asfortranarray(y))
    got = oracle.contract(spec, ext, A, B)
    np.testing.assert_allclose(got.real, f(A.real, B.real) - f(A.imag, B.imag), rtol=0, atol=1e-14)
    np.testing.assert_allclose(got.imag, f(A.real, B.imag) + f(A.imag, B.real), rtol=0, atol=1e-14)


def test_complex_alpha_beta_and_skips():
    rng = np.random.default_rng(16)
    spec, ext = "ab=ai,ib", dict(a=3, b=4, i=5)
    A, B, C0 = crand(rng, "ai", ext, True), crand(rng, "ib", ext, True), crand(rng, "ab", ext, True)
    base = brute(spec, ext, A, B)
    got = oracle.contract(spec, ext, A, B, C=C0.copy(order="F"), alpha=2 - 1j, beta=1j)
    np.testing.assert_array_equal(got, (2 - 1j) * base + 1j * C0)
    # beta == 0 never reads C; alpha == 0 never reads A or B
    nan = np.full_like(C0, complex(np.nan, np.nan))
    np.testing.assert_array_equal(oracle.contract(spec, ext, A, B, C=nan, alpha=1j, beta=0), 1j * base)
    Anan = np.full_like(A, complex(np.nan, np.nan))
    np.testing.assert_array_equal(oracle.contract(spec, ext, Anan, B, C=C0.copy(order="F"), alpha=0, beta=-1j),
                                  -1j * C0)


def test_strided_views_and_zero_extents():
    rng = np.random.default_rng(17)
    spec, ext = "abc=ai,ibc", dict(a=3, b=2, c=2, i=4)
    big = crand(rng, "xy", dict(x=7, y=9))
    A = big[1::2, 1:9:2]                             # non-unit strides in both axes
    B = crand(rng, "ibc", ext)
    np.testing.assert_allclose(oracle.contract(spec, ext, A, B), np.einsum("ai,ibc->abc", A, B), atol=1e-14)
    ext0 = dict(ext, i=0)
    out = oracle.contract(spec, ext0, np.zeros((3, 0), np.complex128, order="F"),
                          np.zeros((0, 2, 2), np.complex128, order="F"))
    assert out.shape == (3, 2, 2) and np.all(out == 0)


def test_error_metric_counts_imaginary_parts():
    ref = np.array([3 + 4j, 0j])
    assert oracle.normwise_rel_err(ref, ref) == 0.0
    assert oracle.normwise_rel_err(np.array([3 + 3j, 0j]), ref) == pytest.approx(1 / 5)
    assert oracle.normwise_rel_err(np.array([3 + 4j, 1j]), ref) == pytest.approx(1 / 5)
