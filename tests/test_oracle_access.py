"""Pins for the symbolic prediction oracle (Section 3): the paper's worked
example for ca-gemv (sizes, distances, setup list, 5/4-cache cut, prefetch and
prefetch-failure setups) and the invariants the paper states."""
import pytest

from oracle import access as ac, family


def regions(v):
    return [ac.Region(o.tensor, o.letters, o.fixed) for o in v.operands]


def test_worked_example(golden):
    g = golden("access_example.json")
    v = {x.name: x for x in family.enumerate_family(g["spec"])}[g["variant"]]
    ops = regions(v)
    ext = g["extents"]
    for r in ops:
        assert ac.region_size(r, set(), ext) == g["sizes"][r.tensor]
        assert ac.access_distance(r, ops, v.loops, ext) == g["distances"][r.tensor]
    items = [(r.tensor, ac.region_size(r, set(), ext), ac.access_distance(r, ops, v.loops, ext)) for r in ops]
    full = ac.build_setup(items, 1e30)
    assert [list(e) for e in full] == g["setup_full"]
    cut = ac.build_setup(items, g["cache_elems"])
    assert [list(e) for e in cut] == g["setup_truncated"]
    assert sum(e[2] for e in cut) == g["truncation_limit"] == 5 * g["cache_elems"] // 4
    kinds = {r.tensor: ac.prefetch_kind(r, v.loops, ext, g["line_elems"]) for r in ops}
    assert sorted(t for t, k in kinds.items() if k) == g["prefetched"]
    cls = ac.predict_classes(ops, v.loops, ext, g["cache_elems"], g["line_elems"], stage=4)
    steady = [c for c in cls if c.label == "steady"][0]
    fail = [c for c in cls if c.label == "fail"][0]
    assert steady.setup == g["setup_prefetch"]
    assert [list(e) for e in fail.setup] == g["setup_fail"]
    assert abs(fail.weight - 1.0 / g["fail_period"]) < 1e-15


def test_stage2_is_truncated_list(golden):
    g = golden("access_example.json")
    v = {x.name: x for x in family.enumerate_family(g["spec"])}[g["variant"]]
    cls = ac.predict_classes(regions(v), v.loops, g["extents"], g["cache_elems"], g["line_elems"], stage=2)
    assert len(cls) == 1 and [list(e) for e in cls[0].setup] == g["setup_truncated"]
    cls1 = ac.predict_classes(regions(v), v.loops, g["extents"], g["cache_elems"], g["line_elems"], stage=1)
    assert cls1[0].setup == [] and cls1[0].weight == 1.0


@pytest.mark.parametrize("spec", ["abc=ai,ibc", "abc=ija,jbic", "a=iaj,ji"])
def test_invariants_all_variants(spec):
    """Before the cut, the sizes to the right of each operand add up to its
    distance (when no remote size had to be clamped); class weights sum to 1."""
    ext = {ch: n for ch, n in zip("abcdij", (40, 30, 20, 10, 8, 6))}
    for v in family.enumerate_family(spec):
        ops = regions(v)
        items = [(r.tensor, ac.region_size(r, set(), ext), ac.access_distance(r, ops, v.loops, ext)) for r in ops]
        order = sorted(items, key=lambda t: -t[2])
        clamped = any(order[k][2] - order[k + 1][2] - order[k + 1][1] < 0 for k in range(len(order) - 1))
        seq = ac.build_setup(items, 1e30)
        if not clamped:
            for pos, e in enumerate(seq):
                if e[0] == "op":
                    d = [it[2] for it in items if it[0] == e[1]][0]
                    assert sum(x[2] for x in seq[pos + 1:]) == d, v.name
        for st in range(1, 6):
            cls = ac.predict_classes(ops, v.loops, ext, 1000.0, 16, stage=st)
            assert abs(sum(c.weight for c in cls) - 1.0) < 1e-12, (v.name, st)
            for c in cls:
                assert sum(e[2] for e in c.setup) <= 1250.0 + 1e-9


def test_case_rules_on_other_printed_algorithms():
    """Section 3.2's three cases on the ger examples of Section 3.3/3.5."""
    ext = dict(a=400, b=400, c=400, i=8)
    vs = {x.name: x for x in family.enumerate_family("abc=ai,ibc")}
    v = vs["bi-ger"]                       # for b, for i: C[:,b,:] += A[:,i] B[i,b,:]^T
    ops = regions(v)
    kinds = {r.tensor: ac.prefetch_kind(r, v.loops, ext, 8) for r in ops}
    # A[:,i]: i indexes its second axis and the first is whole -> streamed;
    # B[i,b,:]: i indexes its first axis -> shares cache lines (Section 3.3 example)
    assert kinds == {"A": "stream", "B": "line", "C": None}
    d = {r.tensor: ac.access_distance(r, ops, v.loops, ext) for r in ops}
    assert d["C"] == 0                                  # C[:,b,:] does not vary with i
    assert d["A"] == 400 * 8 + 8 * 400 + 400 * 400       # A[:,:], B[:,b,:], C[:,b,:]
    v = vs["ci-ger"]                       # first iteration of i: C[:,:,c] changes (Section 3.5)
    cls = ac.predict_classes(regions(v), v.loops, ext, 786432, 8, stage=5)
    first = [c for c in cls if c.label == "first@i"][0]
    assert abs(first.weight - (1 / 8) * (1 - 1 / 400)) < 1e-15 or abs(first.weight - 1 / 8) < 1e-15
    assert any(c.label.startswith("first") for c in cls)


def test_root_gap_only_where_the_walk_reaches_the_root(golden):
    """Section 3.2's third case: in the worked example only C's walk reaches the
    root (its set M holds every operand whole), so a caller's gap moves C's
    distance by exactly the gap and leaves A's and B's (case 1) alone."""
    g = golden("access_example.json")
    v = {x.name: x for x in family.enumerate_family(g["spec"])}[g["variant"]]
    ops = regions(v)
    ext = g["extents"]
    at_root = {t for t, m in g["M_sets"].items() if m and all(":" in x and "c" not in x.split("[")[1] for x in m)}
    assert at_root == {"C"}
    for gap in (0, 1, 1000, 10 ** 9):
        for r in ops:
            want = g["distances"][r.tensor] + (gap if r.tensor in at_root else 0)
            assert ac.access_distance(r, ops, v.loops, ext, root_gap=gap) == want


def test_large_root_gap_makes_an_operand_cold():
    """A gap beyond 5/4 of the cache pushes an operand whose walk reaches the
    root out of the cut setup list; a gap of 0 keeps the paper's list."""
    spec, ext = "abc=ai,ibc", dict(a=40, b=30, c=20, i=8)
    cache = 40000.0                  # the three whole tensors (29,120) fit in 5/4 of it
    checked = 0
    for v in family.enumerate_family(spec):
        ops = regions(v)
        for r in ops:
            d0 = ac.access_distance(r, ops, v.loops, ext)
            d1 = ac.access_distance(r, ops, v.loops, ext, root_gap=10 ** 6)
            if d1 == d0 or d0 + ac.region_size(r, set(), ext) > 1.25 * cache:
                continue
            base = ac.predict_classes(ops, v.loops, ext, cache, 8, stage=2)[0].setup
            cold = ac.predict_classes(ops, v.loops, ext, cache, 8, stage=2, root_gaps={r.tensor: 10 ** 6})[0].setup
            assert ["op", r.tensor, ac.region_size(r, set(), ext)] in [list(e) for e in base], v.name
            assert r.tensor not in [e[1] for e in cold], v.name
            checked += 1
    assert checked >= 20


def test_chain_root_gaps_hand_worked():
    # two contractions, T = A B then D = T E (ids 1..5, bytes)
    two = [[(1, 100), (2, 1000), (3, 5000)], [(3, 5000), (4, 300), (5, 700)]]
    assert ac.chain_root_gaps(two) == [[1000, 1000, 0], [0, 1100, 1100]]
    # three contractions over six tensors of 10..60 bytes
    s = {i: 10 * i for i in range(1, 7)}
    three = [[(1, s[1]), (2, s[2]), (3, s[3])], [(3, s[3]), (4, s[4]), (5, s[5])], [(5, s[5]), (1, s[1]), (6, s[6])]]
    assert ac.chain_root_gaps(three) == [[0, 150, 110], [0, 90, 30], [0, 70, 90]]
    # one contraction alone is the paper's assumption: nothing in between
    assert ac.chain_root_gaps([[(1, 8), (2, 8), (3, 8)]]) == [[0, 0, 0]]
