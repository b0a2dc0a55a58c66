"""Pins for the FP64 loop-nest oracle (Section 1 definition) against things
other than itself: brute force, textbook BLAS reductions, identity tensors,
linearity, index relabelling/permutation symmetry, degenerate extents and the
classical dot-product error bound."""
import itertools

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

PATTERNS = ["abc=ai,ibc", "abc=ija,jbic", "ab=iaj,jbi", "abcd=ai,ibcd", "a=iaj,ji"]


def rand_tensor(rng, letters, ext, integer=False):
    shape = [ext[ch] for ch in letters]
    if integer:
        x = rng.integers(-2, 3, size=shape).astype(np.float64)
    else:
        x = rng.uniform(-1, 1, size=shape)
    return np.array(x, order="F")          # keeps 0-d tensors 0-d


def brute(spec, ext, A, B):
    """Sum over every assignment of every index: C[f] += A[.]B[.]."""
    sa, sb, sc = oracle.split_spec(spec)
    letters = sorted(set(sa + sb + sc))
    C = np.zeros([ext[ch] for ch in sc])
    for vals in itertools.product(*[range(ext[ch]) for ch in letters]):
        env = dict(zip(letters, vals))
        C[tuple(env[ch] for ch in sc)] += A[tuple(env[ch] for ch in sa)] * B[tuple(env[ch] for ch in sb)]
    return C


@pytest.mark.parametrize("spec", PATTERNS)
@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_brute_force_integer_exact(spec, n):
    rng = np.random.default_rng(100 + n)
    letters = set(spec.replace("=", "").replace(",", ""))
    ext = {ch: int(rng.integers(max(0, n - 1), n + 2)) for ch in letters}
    sa, sb, sc = oracle.split_spec(spec)
    A, B = rand_tensor(rng, sa, ext, True), rand_tensor(rng, sb, ext, True)
    C = oracle.contract(spec, ext, A, B)
    np.testing.assert_array_equal(C, brute(spec, ext, A, B))


@given(st.data())
@settings(max_examples=40, deadline=None)
def test_random_specs_vs_brute(data):
    """Random two-operand contractions of up to 5 indices (free and contracted)."""
    letters = "abcdeijk"
    n_free_a = data.draw(st.integers(0, 2))
    n_free_b = data.draw(st.integers(0, 2))
    n_con = data.draw(st.integers(0, 2))
    pool = data.draw(st.permutations(list(letters)))
    fa, fb, k = pool[:n_free_a], pool[n_free_a:n_free_a + n_free_b], pool[n_free_a + n_free_b:n_free_a + n_free_b + n_con]
    sa = "".join(data.draw(st.permutations(fa + k)))
    sb = "".join(data.draw(st.permutations(fb + k)))
    sc = "".join(data.draw(st.permutations(fa + fb)))
    spec = f"{sc}={sa},{sb}"
    ext = {ch: data.draw(st.integers(0, 3)) for ch in fa + fb + k}
    rng = np.random.default_rng(data.draw(st.integers(0, 2**31)))
    A, B = rand_tensor(rng, sa, ext, True), rand_tensor(rng, sb, ext, True)
    np.testing.assert_array_equal(oracle.contract(spec, ext, A, B), brute(spec, ext, A, B))


def test_textbook_gemm_gemv_dot():
    rng = np.random.default_rng(7)
    M, N, K = 7, 5, 9
    A = np.asfortranarray(rng.integers(-3, 4, (M, K)).astype(float))
    B = np.asfortranarray(rng.integers(-3, 4, (K, N)).astype(float))
    C = oracle.contract("ab=ai,ib", dict(a=M, b=N, i=K), A, B)
    ref = np.zeros((M, N))
    for r in range(M):
        for q in range(N):
            for p in range(K):
                ref[r, q] += A[r, p] * B[p, q]
    np.testing.assert_array_equal(C, ref)
    x = np.asfortranarray(B[:, 0].copy())
    y = oracle.contract("a=ai,i", dict(a=M, i=K), A, x)
    np.testing.assert_array_equal(y, A @ x)
    d = oracle.contract("=i,i", dict(i=K), x, x)
    assert d.shape == () and float(d) == float(np.dot(x, x))
    # a third-party routine on integer data, where every order is exact
    A4 = rand_tensor(rng, "ija", dict(i=3, j=4, a=5), True)
    B4 = rand_tensor(rng, "jbic", dict(j=4, b=2, i=3, c=3), True)
    C4 = oracle.contract("abc=ija,jbic", dict(i=3, j=4, a=5, b=2, c=3), A4, B4)
    np.testing.assert_array_equal(C4, np.einsum("ija,jbic->abc", A4, B4))


def test_identity_tensors():
    rng = np.random.default_rng(3)
    # A[a,i] = delta_ai gives C = B for abc=ai,ibc
    n, b, c = 6, 4, 5
    A = np.asfortranarray(np.eye(n))
    B = rand_tensor(rng, "ibc", dict(i=n, b=b, c=c))
    np.testing.assert_array_equal(oracle.contract("abc=ai,ibc", dict(a=n, i=n, b=b, c=c), A, B), B)
    # A[i,j,a] = delta_ia delta_{j,j0} gives C[a,b,c] = B[j0,b,a,c] (permuted strides)
    i = 5
    j, j0 = 4, 2
    A = np.zeros((i, j, i), order="F")
    for t in range(i):
        A[t, j0, t] = 1.0
    B = rand_tensor(rng, "jbic", dict(j=j, b=3, i=i, c=2))
    C = oracle.contract("abc=ija,jbic", dict(i=i, j=j, a=i, b=3, c=2), A, B)
    np.testing.assert_array_equal(C, np.transpose(B[j0], (1, 0, 2)))


@pytest.mark.parametrize("spec", PATTERNS)
def test_linearity_and_alpha_beta(spec):
    rng = np.random.default_rng(11)
    letters = set(spec.replace("=", "").replace(",", ""))
    ext = {ch: int(rng.integers(1, 4)) for ch in letters}
    sa, sb, sc = oracle.split_spec(spec)
    A1, A2 = rand_tensor(rng, sa, ext, True), rand_tensor(rng, sa, ext, True)
    B1, B2 = rand_tensor(rng, sb, ext, True), rand_tensor(rng, sb, ext, True)
    f = lambda A, B, **kw: oracle.contract(spec, ext, A, B, **kw)
    np.testing.assert_array_equal(f(A1 + A2, B1), f(A1, B1) + f(A2, B1))
    np.testing.assert_array_equal(f(A1, B1 - B2), f(A1, B1) - f(A1, B2))
    C0 = rand_tensor(rng, sc, ext, True)
    got = f(A1, B1, C=C0.copy(order="F"), alpha=0.5, beta=-4.0)
    np.testing.assert_array_equal(got, 0.5 * f(A1, B1) - 4.0 * C0)
    # alpha = 0 reads neither input: NaNs there must not reach C
    An = np.full_like(A1, np.nan)
    got = f(An, B1, C=C0.copy(order="F"), alpha=0.0, beta=2.0)
    np.testing.assert_array_equal(got, 2.0 * C0)
    # beta = 0 does not read C
    Cn = np.full_like(C0, np.nan)
    np.testing.assert_array_equal(f(A1, B1, C=Cn, alpha=1.0, beta=0.0), f(A1, B1))


def test_relabel_permute_swap():
    rng = np.random.default_rng(5)
    ext = dict(i=3, j=4, a=5, b=2, c=3)
    A = rand_tensor(rng, "ija", ext, True)
    B = rand_tensor(rng, "jbic", ext, True)
    C = oracle.contract("abc=ija,jbic", ext, A, B)
    # relabel letters
    ren = dict(i="p", j="q", a="x", b="y", c="z")
    ext2 = {ren[k]: v for k, v in ext.items()}
    np.testing.assert_array_equal(oracle.contract("xyz=pqx,qypz", ext2, A, B), C)
    # permute A's modes together with its strides (same memory, new spec order)
    Ap = np.transpose(A, (2, 0, 1))            # axes a, i, j: a view with permuted strides
    np.testing.assert_array_equal(oracle.contract("abc=aij,jbic", ext, Ap, B), C)
    # swap the inputs
    np.testing.assert_array_equal(oracle.contract("abc=jbic,ija", ext, B, A), C)
    # permute C's storage order: compute into a C-ordered output
    Cc = np.zeros((5, 2, 3), order="C")
    np.testing.assert_array_equal(oracle.contract("abc=ija,jbic", ext, A, B, C=Cc), C)
    # a broadcast (stride 0) input equals the materialised one
    Bb = np.broadcast_to(B[:, :, :1, :], B.shape)
    np.testing.assert_array_equal(oracle.contract("abc=ija,jbic", ext, A, Bb),
                                  oracle.contract("abc=ija,jbic", ext, A, np.asfortranarray(Bb)))


def test_zero_extents():
    rng = np.random.default_rng(9)
    ext = dict(a=3, b=2, c=2, i=0)
    A = np.zeros((3, 0), order="F")
    B = np.zeros((0, 2, 2), order="F")
    C0 = rand_tensor(rng, "abc", ext)
    got = oracle.contract("abc=ai,ibc", ext, A, B, C=C0.copy(order="F"), alpha=1.0, beta=3.0)
    np.testing.assert_array_equal(got, 3.0 * C0)
    ext = dict(a=0, b=2, c=2, i=4)
    out = oracle.contract("abc=ai,ibc", ext, np.zeros((0, 4), order="F"), rand_tensor(rng, "ibc", ext))
    assert out.shape == (0, 2, 2)


@pytest.mark.parametrize("bad", ["abc=ai,ib", "abc=aai,ibc", "abc=ai", "aBc=ai,iBc", "abcx=ai,ibc"])
def test_rejects_malformed_specs(bad):
    ext = dict(a=2, b=2, c=2, i=2, x=2, B=2)
    sa, sb, sc = (bad.split("=")[1].split(",") + [""])[:2] + [bad.split("=")[0]]
    with pytest.raises(Exception):
        oracle.contract(bad, ext, np.zeros([2] * len(sa)), np.zeros([2] * len(sb)))


def test_error_bound_against_dot2():
    """|C - C_exact| <= gamma_K |A||B| (Higham, Section 3.1), C_exact from the
    doubled-precision accumulation; and the two differ on real data."""
    rng = np.random.default_rng(13)
    ext = dict(a=16, b=8, c=4, i=512)
    A = rand_tensor(rng, "ai", ext)
    B = rand_tensor(rng, "ibc", ext)
    C = oracle.contract("abc=ai,ibc", ext, A, B)
    Cx = oracle.contract("abc=ai,ibc", ext, A, B, dot2=True)
    absAB = oracle.contract("abc=ai,ibc", ext, np.abs(A), np.abs(B))
    u = 2.0 ** -53
    assert np.all(np.abs(C - Cx) <= oracle.gamma(512, u) * absAB)
    assert np.any(C != Cx)
    # Dot2 is exact on a sum that cancels catastrophically in plain FP64
    x = np.array([1e16, 1.0, -1e16, 1.0], order="F")
    y = np.ones(4, order="F")
    assert float(oracle.contract("=i,i", dict(i=4), x, y, dot2=True)) == 2.0


def test_fixed_summation_order():
    """The contracted sum runs in A's index order, first index fastest: with
    values whose FP64 sum depends on the order, the result equals an explicit
    left-to-right sum in that order."""
    ext = dict(i=3, j=2)
    big = [1e16, 1.0, 1.0, -1e16, 1.0, 1.0]
    A = np.asfortranarray(np.array(big).reshape((3, 2), order="F"))
    B = np.ones((2, 3), order="F")          # B[j, i]
    got = float(oracle.contract("=ij,ji", ext, A, B))
    acc = 0.0
    for j in range(2):
        for i in range(3):
            acc += A[i, j] * 1.0
    assert got == acc


def test_error_metrics():
    C = np.array([3.0, 4.0])
    assert oracle.normwise_rel_err(C, C) == 0.0
    assert abs(oracle.normwise_rel_err(C + np.array([0.3, 0.4]), C) - 0.1) < 1e-15
    assert oracle.componentwise_err(np.array([1.5]), np.array([1.0]), np.array([2.0])) == 0.25
    assert oracle.flops("abc=ai,ibc", dict(a=64, b=64, c=64, i=8)) == 4194304


# Index classes the paper does not define, read as the same sum over every index
# absent from C: batch indices (in A, B and C) and trace indices (one input only).
GENERAL = ["ab=iab,ib", "abc=aic,ibc", "a=iat,i", "ab=ai,ibt", "abc=aict,ibcs", "b=tb,sb"]


@pytest.mark.parametrize("spec", GENERAL)
@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_batch_and_trace_brute_force(spec, n):
    rng = np.random.default_rng(300 + n)
    letters = set(spec.replace("=", "").replace(",", ""))
    ext = {ch: int(rng.integers(max(0, n - 1), n + 2)) for ch in letters}
    sa, sb, sc = oracle.split_spec(spec)
    A, B = rand_tensor(rng, sa, ext, True), rand_tensor(rng, sb, ext, True)
    np.testing.assert_array_equal(oracle.contract(spec, ext, A, B), brute(spec, ext, A, B))


def test_batch_index_is_slicewise_contraction():
    """Each value of a batch index is the paper's contraction of the slices
    (same summation order, so bit-identical on real data)."""
    rng = np.random.default_rng(31)
    ext = dict(a=5, b=4, c=3, i=7)
    A, B = rand_tensor(rng, "aic", ext), rand_tensor(rng, "ibc", ext)
    C = oracle.contract("abc=aic,ibc", ext, A, B, alpha=1.5)
    for c in range(ext["c"]):
        ref = oracle.contract("ab=ai,ib", dict(a=5, b=4, i=7), np.asfortranarray(A[:, :, c]),
                              np.asfortranarray(B[:, :, c]), alpha=1.5)
        np.testing.assert_array_equal(C[:, :, c], ref)


def test_trace_index_is_presummed_operand():
    """A trace index of A equals contracting the summed-out A (integers: exact);
    the same on B's side."""
    rng = np.random.default_rng(32)
    ext = dict(a=6, i=5, t=4, b=3, s=2)
    A, B = rand_tensor(rng, "iat", ext, True), rand_tensor(rng, "ib", ext, True)
    got = oracle.contract("ab=iat,ib", ext, A, B)
    ref = oracle.contract("ab=ia,ib", ext, np.asfortranarray(A.sum(axis=2)), B)
    np.testing.assert_array_equal(got, ref)
    A2, B2 = rand_tensor(rng, "ia", ext, True), rand_tensor(rng, "sib", ext, True)
    got = oracle.contract("ab=ia,sib", ext, A2, B2)
    ref = oracle.contract("ab=ia,ib", ext, A2, np.asfortranarray(B2.sum(axis=0)))
    np.testing.assert_array_equal(got, ref)


@given(st.data())
@settings(max_examples=40, deadline=None)
def test_random_general_specs_vs_brute(data):
    """Random specs with free, contracted, batch and trace indices."""
    letters = "abcdeijkst"
    counts = [data.draw(st.integers(0, 1)) for _ in range(6)]   # fa, fb, k, batch, ta, tb
    pool = data.draw(st.permutations(list(letters)))
    groups, at = [], 0
    for c in counts:
        groups.append(pool[at:at + c])
        at += c
    fa, fb, k, bt, ta, tb = groups
    sa = "".join(data.draw(st.permutations(fa + k + bt + ta)))
    sb = "".join(data.draw(st.permutations(fb + k + bt + tb)))
    sc = "".join(data.draw(st.permutations(fa + fb + bt)))
    spec = f"{sc}={sa},{sb}"
    ext = {ch: data.draw(st.integers(0, 3)) for ch in set(sa + sb + sc)}
    rng = np.random.default_rng(data.draw(st.integers(0, 2**31)))
    A, B = rand_tensor(rng, sa, ext, True), rand_tensor(rng, sb, ext, True)
    np.testing.assert_array_equal(oracle.contract(spec, ext, A, B), brute(spec, ext, A, B))


@pytest.mark.parametrize("spec,ext", [
    ("abc=ai,ibc", dict(a=13, b=7, c=9, i=5)),
    ("abc=ija,jbic", dict(a=6, b=5, c=11, i=3, j=4)),
    ("ab=iaj,jbi", dict(a=9, b=8, i=3, j=5)),
    ("=i,i", dict(i=17)),
    ("abcd=ai,ibcd", dict(a=3, b=4, c=2, d=6, i=3)),
])
def test_threaded_oracle_equals_serial(spec, ext):
    """The CPU-baseline timing's threaded run (C's outermost index over host
    threads) gives the serial oracle's values bit for bit, with alpha and beta,
    for every pattern and a 0-d C."""
    from paper_1409_8608_amd import workloads as wl
    A, B, C0 = wl.tensors(spec, ext, np.random.default_rng(7), with_c=True)
    for alpha, beta in ((1.0, 0.0), (-0.75, 1.5), (0.0, 2.0)):
        r1 = oracle.contract(spec, ext, A, B, C=np.array(C0, order="F"), alpha=alpha, beta=beta)
        for threads in (2, 5):
            rt = oracle.contract(spec, ext, A, B, C=np.array(C0, order="F"), alpha=alpha, beta=beta,
                                 threads=threads)
            np.testing.assert_array_equal(rt, r1)
