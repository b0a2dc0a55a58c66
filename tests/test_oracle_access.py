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


# The worked numbers below are derived by hand from the rules of Sections
# 3.2-3.5 at a = b = c = 400, i = 8, a 64-byte line (8 doubles) and the 6 MB
# cache (786,432 doubles, 5/4 of it 983,040), the paper's example setting.
EXT_400 = dict(a=400, b=400, c=400, i=8)
CACHE_6MB, LINE_8 = 786432, 8


def _ci_ger_first_iteration_problems(acc):
    """Mismatches between module ``acc``'s first-iteration class of ci-ger and
    Section 3.5's example.  ci-ger is: for c, for i: C[:,:,c] += A[:,i] B[i,:,c]^T.
    The class of the first i iteration (the next c iteration) starts the walk at
    loop i with M = {A[:,:], B[:,:,c], C[:,:,c]} (every operand joined across i):
      A[:,:] does not change across c (case 1): distance |M| = 3,200 + 3,200 +
        160,000 = 166,400 -- not 0, so A's prefetch "fails", as the paper says;
      B[:,:,c] and C[:,:,c] change across c (case 2): joined along c, M =
        A[:,:] + B[:,:,:] + C[:,:,:] = 3,200 + 1,280,000 + 64,000,000 =
        65,283,200 at the root (case 3) -- C "refers to a different memory
        location", so its distance is not 0.
    No prefetch emulation: A is accessed whole (400 doubles, not one line).
    Setup list: B 400, C 160,000 (the remote region between two operands at
    the same distance would be negative: dropped), remote 65,283,200 - 166,400
    - 400 = 65,116,400, A 400, remote 166,400; cut from the front to 983,040:
    remote 983,040 - 166,800 = 816,240, A 400, remote 166,400.
    Shares: loop i's first iteration is 1/8 of the invocations; loop c's
    (1/3200, under 1%) has no class of its own and counts in first@i, so
    first@i weighs exactly 1/8 and the steady and failure classes share 7/8
    (7/8 * 7/8 and 7/8 * 1/8: B[i,:,c] shares cache lines along i)."""
    vs = {x.name: x for x in family.enumerate_family("abc=ai,ibc")}
    v = vs["ci-ger"]
    problems = []
    if "".join(v.loops) != "ci":
        return [f"loops {v.loops}"]
    ops = regions(v)
    want = {"A": 166400, "B": 65283200, "C": 65283200}
    for r in ops:
        got = acc.access_distance(r, ops, v.loops, EXT_400, start=1, preset={"i"})
        if got != want[r.tensor]:
            problems.append(f"distance {r.tensor} {got} != {want[r.tensor]}")
    cls = acc.predict_classes(ops, v.loops, EXT_400, 1e30, LINE_8, stage=5)
    first = [c for c in cls if c.label.startswith("first")]
    if [c.label for c in first] != ["first@i"]:
        return problems + [f"first-iteration classes {[c.label for c in first]}"]
    f = first[0]
    if f.weight != 1 / 8:
        problems.append(f"weight {f.weight!r} != 1/8")
    full = [["op", "B", 400], ["op", "C", 160000], ["remote", None, 65116400], ["op", "A", 400],
            ["remote", None, 166400]]
    if [list(e) for e in f.setup] != full:
        problems.append(f"uncut setup {f.setup}")
    cut = acc.predict_classes(ops, v.loops, EXT_400, CACHE_6MB, LINE_8, stage=5)
    fc = [c for c in cut if c.label == "first@i"]
    if not fc or [list(e) for e in fc[0].setup] != [["remote", None, 816240], ["op", "A", 400],
                                                    ["remote", None, 166400]]:
        problems.append(f"cut setup {fc[0].setup if fc else None}")
    w = {c.label: c.weight for c in cut}
    if w.get("steady") != (7 / 8) * (7 / 8) or w.get("fail") != (7 / 8) / 8:
        problems.append(f"steady/fail weights {w}")
    return problems


def test_first_iteration_class_ci_ger():
    assert _ci_ger_first_iteration_problems(ac) == []


def test_first_iteration_pin_catches_planted_mistakes(monkeypatch):
    """Each plausible mistake in the first-iteration walk, planted in the
    oracle (on the CPU), makes the pin above fail."""
    real_distance = ac.access_distance

    def one_loop_out(r, ops, loops, extents, start=None, preset=None, root_gap=0):
        if start is not None and start > 0:          # start at the loop outside, joined across it too
            start -= 1
            preset = set(loops[start:])
        return real_distance(r, ops, loops, extents, start, preset, root_gap)

    def m_not_preloaded(r, ops, loops, extents, start=None, preset=None, root_gap=0):
        return real_distance(r, ops, loops, extents, start, None, root_gap)

    real_first = ac.first_iteration_class

    def prefetch_kept(ops, loops, extents, k, share, cache_elems, gaps, keep_operand_only=False, distance=None):
        c = real_first(ops, loops, extents, k, share, cache_elems, gaps, keep_operand_only, distance)
        pre = {r.tensor: ac.prefetch_access_size(r, extents, LINE_8) for r in ops
               if ac.prefetch_kind(r, loops, extents, LINE_8)}
        c.setup = [(e[0], e[1], pre.get(e[1], e[2]) if e[0] == "op" else e[2]) for e in c.setup]
        return c

    for name, fn in (("access_distance", one_loop_out), ("access_distance", m_not_preloaded),
                     ("first_iteration_class", prefetch_kept)):
        with monkeypatch.context() as m:
            m.setattr(ac, name, fn)
            assert _ci_ger_first_iteration_problems(ac), fn.__name__


def test_prefetch_access_sizes():
    """Section 3.3: a prefetched operand's setup access is limited to one cache
    line along its first axis.  ca-gemv (its second example): C[a,:,c] and
    A[a,:] have extent 1 along their first axis, so they are accessed whole
    (400 and 8), and the reduced list, before it is dropped for holding only
    operand accesses, is C[a,:,c], A[a,:], B[:,:,c] (400, 8, 3,200), in the
    order of their access distances.  bi-ger (its first example): A[:,i] is
    streamed along its 400-long first axis, so its access is one line of 8
    doubles; B[i,b,:] (first-axis extent 1) is whole, 400; C[:,b,:] is not
    prefetched and keeps its 160,000.  Its access distances order the list
    B (65,283,200), A (166,400), C (0)."""
    vs = {x.name: x for x in family.enumerate_family("abc=ai,ibc")}
    v = vs["ca-gemv"]
    ops = regions(v)
    assert {r.tensor: ac.prefetch_access_size(r, EXT_400, LINE_8) for r in ops} == {"A": 8, "B": 3200, "C": 400}
    st = ac.predict_classes(ops, v.loops, EXT_400, CACHE_6MB, LINE_8, stage=3, keep_operand_only=True)
    assert [list(e) for e in st[0].setup] == [["op", "C", 400], ["op", "A", 8], ["op", "B", 3200]]
    v = vs["bi-ger"]
    ops = regions(v)
    sizes = {r.tensor: ac.prefetch_access_size(r, EXT_400, LINE_8) for r in ops}
    assert sizes["A"] == 8 and sizes["B"] == 400
    st = ac.predict_classes(ops, v.loops, EXT_400, CACHE_6MB, LINE_8, stage=3, keep_operand_only=True)
    assert [list(e) for e in st[0].setup] == [["op", "B", 400], ["op", "A", 8], ["op", "C", 160000]]
    # Section 3.4: the failure benchmark drops the line-sharing emulation of
    # B[i,b,:] (back at its access distance), A stays one streamed line:
    # B 400, remote 65,283,200 - 0 - 8, A 8, C 160,000; cut to 983,040:
    # remote 983,040 - 160,008 = 823,032, A 8, C 160,000
    st = ac.predict_classes(ops, v.loops, EXT_400, CACHE_6MB, LINE_8, stage=4)
    fail = [c for c in st if c.label == "fail"][0]
    assert [list(e) for e in fail.setup] == [["remote", None, 823032], ["op", "A", 8], ["op", "C", 160000]]
    assert fail.weight == 1 / 8


def test_prefetch_list_order_pin_catches_operand_order(golden):
    """The printed reduced list of Section 3.3 fixes the order of operands at
    equal distance: ordering ties by operand (A, B, C) instead of by access
    distance gives A, B, C and fails."""
    g = golden("access_example.json")
    v = {x.name: x for x in family.enumerate_family(g["spec"])}[g["variant"]]
    ops = regions(v)
    st = ac.predict_classes(ops, v.loops, g["extents"], g["cache_elems"], g["line_elems"], stage=3,
                            keep_operand_only=True)
    assert [list(e) for e in st[0].setup] == g["setup_prefetch_operands"]
    items = [(r.tensor, ac.prefetch_access_size(r, g["extents"], g["line_elems"]), 0) for r in ops]
    assert [list(e) for e in ac.build_setup(items, g["cache_elems"])] != g["setup_prefetch_operands"]


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


# Algorithms with several statements: the copy members of Section 2 (the walk
# of Section 3.2 over an AST with a copy statement and the kernel).

def test_program_walk_equals_single_kernel_walk_without_copies():
    """With no copy the member's program is one kernel in its loops, and the
    walk over the program gives exactly the single-kernel classes (every stage,
    with and without root gaps) for every copy-free member of six patterns."""
    ext = {ch: n for ch, n in zip("abcdij", (40, 30, 20, 10, 8, 6))}
    n = 0
    for spec in ("abc=ai,ibc", "abc=ija,jbic", "a=iaj,ji", "ab=iaj,jbi", "bac=ai,ibc", "abcd=ai,ibcd"):
        for v in family.enumerate_family(spec):
            if v.copies:
                continue
            for stage in range(1, 6):
                for gaps in (None, {"A": 1000, "B": 0, "C": 50000}):
                    a = ac.predict_classes(regions(v), v.loops, ext, 1000.0, 16, stage=stage, root_gaps=gaps)
                    b = ac.predict_member(v, ext, 1000.0, 16, stage=stage, root_gaps=gaps)
                    assert [(c.label, c.weight, c.setup) for c in a] == [(c.label, c.weight, c.setup) for c in b]
                    n += 1
    assert n > 3000


def test_copy_members_hand_worked():
    """Test 3 (a=b=c=256, i=j=32): A is 262,144 elements, B 67,108,864, C
    16,777,216, the copy buffer A~ = A[i,:,:] 8,192.
    i'c-gemm: for i { A~ := A[i,:,:]; for c { C[:,:,c] += A~^T B[:,:,i,c] } }
      A~: the same buffer in every c iteration (case 1 at loop c): 0.
      B[:,:,i,c]: varies with c, M = {A~, B[:,:,i,:], C}; then the copy, one
        statement earlier in loop i's body, adds A[i,:,:]; varies with i: all of
        it joined along i, the root: |A| + |A~| + |B| + |C| = 84,156,416.
      C[:,:,c]: varies with c, M = {A~, B[:,:,i,:], C}; the copy adds A[i,:,:];
        C[:,:,:] does not vary with i (case 1): 8,192 + 2,097,152 + 16,777,216
        + 8,192 = 18,890,752.
    ci'-gemm: for c { for i { A~ := A[i,:,:]; C[:,:,c] += A~^T B[:,:,i,c] } }
      A~: the copy just before it wrote it: 0.
      B: as above, 84,156,416.
      C[:,:,c]: the copy adds A[i,:,:] and A~; C does not vary with i (case
        1): 16,384 -- where the single-kernel walk, blind to the copy, gives 0.
    Test 2's i'-gemv (a=i=j=n): for i { A~ := A[i,:,:]; C[:] += A~ B[:,i] }:
      A~ 0; B[:,i]: n^3 + 2n^2 + n; C: 2n^2."""
    ext = dict(a=256, b=256, c=256, i=32, j=32)
    vs = {v.name: v for v in family.enumerate_family("abc=ija,jbic")}
    assert ac.kernel_distances(vs["i'c-gemm"], ext) == {"A": 0, "B": 84156416, "C": 18890752}
    assert ac.kernel_distances(vs["ci'-gemm"], ext) == {"A": 0, "B": 84156416, "C": 16384}
    blind = {r.tensor: ac.access_distance(r, regions(vs["ci'-gemm"]), vs["ci'-gemm"].loops, ext)
             for r in regions(vs["ci'-gemm"])}
    assert blind["C"] == 0 and blind["A"] != 0
    n = 64
    v = {x.name: x for x in family.enumerate_family("a=iaj,ji")}["i'-gemv"]
    assert ac.kernel_distances(v, dict(a=n, i=n, j=n)) == {"A": 0, "B": n ** 3 + 2 * n ** 2 + n, "C": 2 * n * n}


def test_copy_member_first_iteration_and_setup():
    """ci'-gemm's first iteration of loop i (weight 1/32; loop c's 1/8192 share
    has no class of its own): the walk starts at loop i with M = {A[:,:,:],
    A~, B[:,:,:,c], C[:,:,c]} (262,144 + 8,192 + 262,144 + 65,536 = 598,016):
    A~ does not vary with c (598,016), B and C vary with c and reach the root
    (84,156,416).  Its steady setup (cache of 10^9 elements, no cut) lists B,
    C and A~ by distance: B 8,192, remote 84,156,416 - 16,384 - 65,536,
    C 65,536, remote 16,384 - 0 - 8,192, A~ 8,192 (A~ is never prefetched: no
    loop changes it)."""
    ext = dict(a=256, b=256, c=256, i=32, j=32)
    v = {x.name: x for x in family.enumerate_family("abc=ija,jbic")}["ci'-gemm"]
    assert ac.kernel_distances(v, ext, start=1) == {"A": 598016, "B": 84156416, "C": 84156416}
    cls = ac.predict_member(v, ext, 1e9, 16, stage=5)
    first = [c for c in cls if c.label.startswith("first")]
    assert [c.label for c in first] == ["first@i"] and first[0].weight == 1 / 32
    st = ac.predict_member(v, ext, 1e9, 16, stage=2)[0].setup
    assert [list(e) for e in st] == [["op", "B", 8192], ["remote", None, 84156416 - 16384 - 65536],
                                     ["op", "C", 65536], ["remote", None, 16384 - 8192], ["op", "A", 8192]]
