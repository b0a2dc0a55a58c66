"""Pins for the family oracle (Section 2): the printed counts, legend names and
numbers, Table 1 pairs, printed operand slices and copy placement; and the
interpreter: every generated variant, run literally as loops of BLAS calls,
equals the plain contraction bit for bit on integer data."""
import numpy as np
import pytest

import oracle
from oracle import family, interp

FIVE = ["abc=ai,ibc", "abc=ija,jbic", "ab=iaj,jbi", "abcd=ai,ibcd", "a=iaj,ji"]


def test_counts(golden):
    g = golden("family_counts.json")
    for spec, want in g.items():
        if spec.startswith("_"):
            continue
        assert family.counts(spec) == want, spec


def test_derived_counts_other_patterns():
    # same rule on the two remaining batch patterns (derived, not printed)
    assert family.counts("ab=iaj,jbi")["total"] == 36
    assert family.counts("abcd=ai,ibcd") == dict(dot=24, axpy=96, gemv=24, ger=18, gemm=6, total=168)


def test_legend_names_and_numbers(golden):
    g = golden("family_names.json")
    for spec, table in g.items():
        if spec.startswith("_"):
            continue
        by_num = {v.number: v.name for v in family.enumerate_family(spec)}
        for num, name in table.items():
            assert by_num[int(num)] == name, (spec, num)


def test_printed_operand_slices(golden):
    g = golden("printed_algorithms.json")
    for spec, algs in g.items():
        if spec.startswith("_") or spec == "table1":
            continue
        vs = {v.name: v for v in family.enumerate_family(spec)}
        for name, want in algs.items():
            v = vs[name]
            pats = {op.tensor: op.pattern() for op in v.operands}
            for t in "ABC":
                assert pats[t] == want[t], (spec, name, t)
            assert sorted(t for t, _ in v.copies) == sorted(want["copies"]), (spec, name)
            assert "".join(v.loops) == want["loops"], (spec, name)
    t1 = g["table1"]
    vs = {v.name: v for v in family.enumerate_family("abc=ai,ibc")}
    for name, want in t1.items():
        if name.startswith("_"):
            continue
        v = vs[name]
        assert sorted(v.kept) == sorted(want["kernel_indices"])
        assert "".join(v.loops) == want["sliced"]


def test_copy_placement_and_counts():
    vs = family.enumerate_family("abc=ija,jbic")
    assert all(v.copies for v in vs if v.kernel == "gemm")
    assert sum(1 for v in vs if v.kernel == "gemv" and v.copies) == 18
    assert not any(v.copies for v in vs if v.kernel in ("dot", "axpy", "ger"))
    assert not any(v.copies for v in family.enumerate_family("abc=ai,ibc"))
    # a copy is hoisted out of the loop it does not depend on (i'c vs ci')
    by = {v.name: v for v in vs}
    assert by["i'c-gemm"].copies == (("A", 0),) and by["ci'-gemm"].copies == (("A", 1),)
    # with explicit strides the unit-stride axis decides: make A's 'a' axis unit stride
    vs2 = {v.name: v for v in family.enumerate_family("abc=ija,jbic", strides={"A": (32, 1024 * 32, 1)})}
    assert "ic-gemm" in vs2 and not vs2["ic-gemm"].copies


@pytest.mark.parametrize("spec", FIVE)
def test_every_variant_equals_contraction(spec):
    rng = np.random.default_rng(17)
    letters = sorted(set(spec.replace("=", "").replace(",", "")))
    ext = {ch: int(v) for ch, v in zip(letters, rng.integers(2, 4, len(letters)))}
    sa, sb, sc = oracle.split_spec(spec)
    A = np.asfortranarray(rng.integers(-2, 3, [ext[c] for c in sa]).astype(float))
    B = np.asfortranarray(rng.integers(-2, 3, [ext[c] for c in sb]).astype(float))
    ref = oracle.contract(spec, ext, A, B)
    for v in family.enumerate_family(spec):
        C = np.zeros([ext[c] for c in sc], order="F")
        interp.run_variant(v, spec, ext, A, B, C)
        np.testing.assert_array_equal(C, ref, err_msg=f"{spec} {v.name}")


def test_misplaced_copy_is_caught():
    """A copy hoisted above a loop its slice depends on feeds a stale slice."""
    import dataclasses
    spec = "abc=ija,jbic"
    ext = dict(i=2, j=2, a=2, b=2, c=3)
    rng = np.random.default_rng(1)
    A = np.asfortranarray(rng.integers(-2, 3, (2, 2, 2)).astype(float))
    B = np.asfortranarray(rng.integers(-2, 3, (2, 2, 2, 3)).astype(float))
    v = {x.name: x for x in family.enumerate_family(spec)}["cj'-gemm"]
    bad = dataclasses.replace(v, copies=(("B", 0),))      # copy at c, but it depends on j
    with pytest.raises(AssertionError):
        interp.run_variant(bad, spec, ext, A, B, np.zeros((2, 2, 3), order="F"))


@pytest.mark.parametrize("spec", ["bac=ai,ibc", "bca=ija,jbic", "bacd=ai,ibcd"])
def test_members_copying_c_equal_contraction(spec):
    """Specs whose C does not start with a kept index of every ger/gemm member:
    those members copy C's slice before the call and back after it (Section 2,
    copies "prior and/or after" the call); every member, copies of C included,
    equals the plain contraction on integer data."""
    rng = np.random.default_rng(23)
    letters = sorted(set(spec.replace("=", "").replace(",", "")))
    ext = {ch: int(v) for ch, v in zip(letters, rng.integers(2, 4, len(letters)))}
    sa, sb, sc = oracle.split_spec(spec)
    A = np.asfortranarray(rng.integers(-2, 3, [ext[c] for c in sa]).astype(float))
    B = np.asfortranarray(rng.integers(-2, 3, [ext[c] for c in sb]).astype(float))
    ref = oracle.contract(spec, ext, A, B)
    fam = family.enumerate_family(spec)
    with_c = [v for v in fam if any(t == "C" for t, _ in v.copies)]
    assert len(with_c) >= 3
    for v in fam:
        C = np.zeros([ext[c] for c in sc], order="F")
        interp.run_variant(v, spec, ext, A, B, C)
        np.testing.assert_array_equal(C, ref, err_msg=f"{spec} {v.name}")
