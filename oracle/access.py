"""Symbolic half of the performance prediction of Section 3 -- TEST
INFRASTRUCTURE ONLY (oracle).

Follows the paper's steps in its order and notation, for the single-kernel loop
nests the family produces (Section 3.2 restricts itself to those):

Access distance (Section 3.2).  For an operand Op of the kernel, walk from the
kernel outwards through the surrounding loops with an initially empty set M:
  1. Op does not vary across the surrounding loop -> stop; the distance is the
     size of M.
  2. Op varies across it -> add all kernel operands to M, joined along every
     loop passed so far (a joined axis becomes ':'), and go up one level.
  3. The root is reached -> the distance is the size of M (the contraction is
     assumed to run repeatedly, nothing else in between).
All operands are distinct tensors here, so |M| is the sum of region sizes.

Setup list (Section 3.2).  Operands sorted by decreasing distance, each followed
by a remote region [r] so that the sizes to the right of an operand add up to
its distance; the last operand is followed by a remote region of its own
distance.  If the list is longer than 5/4 of the cache it is cut from the front
to exactly that length (a cut remote region shrinks; a cut operand is replaced
by a remote region of the part that is kept).  Negative remote sizes are
clamped to 0 and zero-sized remote regions are dropped.

Prefetching (Section 3.3).  Op is prefetched when it varies across the directly
surrounding loop and that loop indexes Op's first axis, or its second axis while
the first is kept whole or fits in one cache line.  A prefetched operand gets
distance 0 and its setup access is limited to one cache line along its first
axis.  A setup made only of operand accesses is dropped (the repetitions of the
benchmark already touch every operand).

Prefetch failures (Section 3.4).  Operands prefetched because the innermost
loop indexes their first axis (line sharing) miss once per cache line, i.e. once
in every L/e iterations (L line bytes, e element bytes).  A second benchmark
without their prefetch emulation takes that share of the steady invocations.

First iterations (Section 3.5).  The first iteration of the innermost loop gets
its own benchmark; an outer loop gets one too when the invocations at which it
and every loop inside it are in their first iteration exceed 1% of all
invocations.  Its distances are found by starting the walk at that loop with M
already holding every operand joined across it and all loops inside it; it uses
no prefetch emulation.  Invocations at the first iteration of a loop without its
own class are counted in the nearest inner class that has one.

Readings where the paper leaves a choice: the prefetch distance is 0 (its worked
example); line failures split only the steady class; a loop nest without loops
gives every operand distance 0.  Operands at equal distance keep the order of
the access-distance list (Section 3.3 folds the prefetch distances into that
list, and its example lists C[a,:,c], A[a,:], B[:,:,c] in the order of their
access distances); operands at equal access distance are taken in the order
A, B, C.

Root precondition (case 3 made explicit).  At the root the paper assumes the
contraction runs again and again with nothing in between, because it cannot
know the surrounding program.  A caller who does know it states, per operand,
how many elements of other data the program touches between the operand's
previous use and this run (its gap); the distance at the root is then |M| plus
that gap.  Gaps of 0 are the paper's assumption.  For a chain of contractions
run in order, again and again, with tensors named by ids, the gap of an operand
is the total size of the distinct tensors that the contractions run since the
operand was last used access, leaving out the tensors of the contraction being
predicted (its own operands are in M already); if no other contraction uses
the tensor, "since it was last used" is the previous run of this contraction.
"""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class Region:
    tensor: str
    letters: str
    fixed: tuple     # per axis: True if fixed by a loop index


def region_size(r: Region, joined: set, extents: dict) -> int:
    n = 1
    for ch, f in zip(r.letters, r.fixed):
        if (not f) or ch in joined:
            n *= int(extents[ch])
    return n


def varies(r: Region, loop: str, joined: set) -> bool:
    """Does operand r (already joined across ``joined``) depend on ``loop``?"""
    return any(f and ch == loop and ch not in joined for ch, f in zip(r.letters, r.fixed))


def access_distance(op: Region, ops, loops, extents: dict, start: int | None = None,
                    preset: set | None = None, root_gap: int = 0) -> int:
    """Distance of ``op`` for a kernel nested in ``loops`` (outermost first).

    ``start``/``preset`` implement the first-iteration variant: the walk starts
    at loop index ``start`` (it and the loops inside it already joined).
    ``root_gap`` is added when the walk reaches the root (case 3)."""
    joined = set(preset or ())
    pos = len(loops) - 1 if start is None else start - 1
    at_root = True
    while pos >= 0:
        loop = loops[pos]
        if not varies(op, loop, joined):
            at_root = False
            break                                   # case 1
        joined.add(loop)                            # case 2
        pos -= 1
    gap = int(root_gap) if at_root else 0           # case 3: the caller's precondition
    if not joined:
        return gap
    return sum(region_size(r, joined, extents) for r in ops) + gap


def chain_root_gaps(chain):
    """Root gaps, in bytes, for a chain of contractions run in order, again and
    again.  ``chain``: one entry per contraction, a list of three (tensor_id,
    bytes) pairs for A, B and C.  Returns one [gap_A, gap_B, gap_C] per
    contraction."""
    n = len(chain)
    size = {}
    for ops in chain:
        for tid, nbytes in ops:
            size[tid] = max(size.get(tid, 0), int(nbytes))
    out = []
    for j, ops in enumerate(chain):
        own = {tid for tid, _ in ops}
        gaps = []
        for tid, _ in ops:
            seen = set()
            for back in range(1, n + 1):            # contractions run since tid was last used
                k = (j - back) % n
                if k == j or tid in {t for t, _ in chain[k]}:
                    break
                seen |= {t for t, _ in chain[k]}
            gaps.append(sum(size[t] for t in seen - own))
        out.append(gaps)
    return out


def build_setup(items, cache_elems: float):
    """items: list of (name, size, distance).  Returns the setup list as
    [('op', name, size) | ('remote', None, size)], applying the 5/4 cut."""
    order = sorted(items, key=lambda t: -t[2])
    seq = []
    for k, (name, size, d) in enumerate(order):
        seq.append(["op", name, size])
        if k + 1 < len(order):
            r = d - order[k + 1][2] - order[k + 1][1]
        else:
            r = d
        seq.append(["remote", None, max(0, r)])
    seq = [e for e in seq if not (e[0] == "remote" and e[2] == 0)]
    limit = 5 * cache_elems / 4
    total = sum(e[2] for e in seq)
    if total > limit:
        kept, acc = [], 0
        for e in reversed(seq):
            if acc + e[2] <= limit:
                kept.append(e)
                acc += e[2]
            else:
                rest = int(limit - acc)
                if rest > 0:
                    kept.append(["remote", None, rest])
                break
        seq = list(reversed(kept))
    return [tuple(e) for e in seq]


def only_operands(setup) -> bool:
    return all(e[0] == "op" for e in setup)


def prefetch_kind(op: Region, loops, extents: dict, line_elems: int):
    """None, 'line' (innermost loop indexes the first axis: cache-line sharing)
    or 'stream' (it indexes the second axis, the first being whole or within
    one line)."""
    if not loops:
        return None
    inner = loops[-1]
    if not varies(op, inner, set()):
        return None
    if op.letters and op.letters[0] == inner:
        return "line"
    if len(op.letters) >= 2 and op.letters[1] == inner:
        first_whole = not op.fixed[0]
        first_small = (not op.fixed[0] and int(extents[op.letters[0]]) <= line_elems) or op.fixed[0]
        if first_whole or first_small:
            return "stream"
    return None


def prefetch_access_size(op: Region, extents: dict, line_elems: int) -> int:
    """One cache line along the first axis, everything else of the operand."""
    n = 1
    for ax, (ch, f) in enumerate(zip(op.letters, op.fixed)):
        e = 1 if f else int(extents[ch])
        if ax == 0:
            e = min(e, line_elems)
        n *= e
    return n


@dataclass
class BenchClass:
    label: str          # 'steady', 'fail', 'first@<loop>'
    weight: float       # share of all kernel invocations
    setup: list         # setup list


def _name(r: Region) -> str:
    """The kernel operand slot ('A', 'B', 'C') of a region (a copy's buffer X~ is X's slot)."""
    return r.tensor.rstrip("~")


def first_iteration_class(ops, loops, extents: dict, k: int, share: float, cache_elems: float,
                          gaps: dict, keep_operand_only: bool = False, distance=None) -> BenchClass:
    """Class of the first iteration of loop ``k`` (Section 3.5): the walk starts
    at that loop with M holding every kernel operand joined across it and the
    loops inside it; every operand is accessed whole (no prefetch emulation).
    ``distance(region, start, gap)`` is the walk (default: the single-kernel one)."""
    if distance is None:
        distance = lambda r, start, gap: access_distance(r, ops, loops, extents, start=start,
                                                         preset=set(loops[start:]) if start is not None else None,
                                                         root_gap=gap)
    items = []
    for r in ops:
        d = distance(r, k, gaps[_name(r)])
        items.append((_name(r), region_size(r, set(), extents), d))
    st = build_setup(items, cache_elems)
    return BenchClass(f"first@{loops[k]}", share, st if keep_operand_only or not only_operands(st) else [])


def predict_classes(ops, loops, extents: dict, cache_elems: float, line_elems: int,
                    stage: int = 5, root_gaps: dict | None = None, keep_operand_only: bool = False,
                    distance=None):
    """Benchmark classes with their shares of the invocations, for prediction
    stage 1 (repeated execution) .. 5 (first iterations separate).
    ``root_gaps`` maps an operand's tensor name to its root gap (elements).
    ``keep_operand_only`` keeps setup lists made only of operand accesses
    (normally dropped: the repetitions already touch every operand), so that
    they can be inspected.  ``distance(region, start, gap)`` is the walk
    (default: the single-kernel walk over ``ops``; ``predict_member`` passes
    the walk of the member's whole program)."""
    names = [_name(r) for r in ops]
    sizes = [region_size(r, set(), extents) for r in ops]
    gaps = {n: int((root_gaps or {}).get(n, 0)) for n in names}
    if stage == 1:
        return [BenchClass("steady", 1.0, [])]
    if distance is None:
        distance = lambda r, start, gap: access_distance(r, ops, loops, extents, start=start,
                                                         preset=set(loops[start:]) if start is not None else None,
                                                         root_gap=gap)
    dist = [distance(r, None, gaps[n]) for r, n in zip(ops, names)]
    kinds = [prefetch_kind(r, loops, extents, line_elems) if stage >= 3 else None for r in ops]
    # the access-distance list's order (ties: A, B, C); later stages keep it for ties
    order = sorted(range(len(ops)), key=lambda t: -dist[t])

    def setup_with(prefetched):
        items = []
        for t in order:
            if prefetched[t]:
                items.append((names[t], prefetch_access_size(ops[t], extents, line_elems), 0))
            else:
                items.append((names[t], sizes[t], dist[t]))
        st = build_setup(items, cache_elems)
        return st if keep_operand_only or not only_operands(st) else []

    steady_setup = setup_with([k is not None for k in kinds])
    classes = []
    n_inner = int(extents[loops[-1]]) if loops else 1
    steady_share = 1.0 - (1.0 / n_inner if (stage >= 5 and loops) else 0.0)
    if stage >= 4 and any(k == "line" for k in kinds):
        period = line_elems
        fail_setup = setup_with([k == "stream" for k in kinds])
        classes.append(BenchClass("steady", steady_share * (period - 1) / period, steady_setup))
        classes.append(BenchClass("fail", steady_share / period, fail_setup))
    else:
        classes.append(BenchClass("steady", steady_share, steady_setup))
    if stage >= 5 and loops:
        # share of invocations at which loops[k:] are all in their first iteration
        n = len(loops)
        first_share = [0.0] * n
        for k in range(n):
            s = 1.0
            for m in range(k, n):
                s /= int(extents[loops[m]])
            first_share[k] = s
        own = [k for k in range(n) if k == n - 1 or first_share[k] > 0.01]
        for k in sorted(own, reverse=True):
            outer = [o for o in own if o < k]
            nxt = max(outer) if outer else None
            share = first_share[k] - (first_share[nxt] if nxt is not None else 0.0)
            classes.append(first_iteration_class(ops, loops, extents, k, share, cache_elems, gaps,
                                                 keep_operand_only, distance))
    return classes


# ---------------------------------------------------------------------------
# Algorithms with several statements (Section 3.2: the back-traversal "allows
# for any combinations of loops and multiple kernels within the AST").
#
# A family member with copies is such an AST: a copy statement X~ := X[slice]
# sits at the head of the body of the loop that the slice depends on most
# deeply (before all loops for a slice fixed by none), the kernel works on the
# copy X~ (one buffer, reused in every iteration), and a copy of C is written
# back after the loops inside its level.  The walk of an operand Op of a
# statement S goes backwards through the program from S:
#   - earlier statements of the same loop body (this iteration): if one
#     accesses Op's tensor, Op's previous access is found and the walk stops;
#     otherwise all its regions, joined along the loops inside it, go into M;
#   - then the enclosing loop L:
#       case 1, Op does not vary across L: Op's previous access was in the
#         previous iteration of L; the statements after S's position in L's
#         body ran after it: they are walked backwards from the end of the
#         body, with the same stop rule, and the walk ends;
#       case 2, Op varies across L: every region of L's body, joined along L
#         and the loops inside it, goes into M, Op is joined along L, and the
#         walk continues one level up with L in the place of S;
#   - at the root (case 3), the distance is |M| plus the caller's gap.
# For a single statement this is exactly the walk above.  M holds one region
# per tensor: two regions of a tensor are merged into the smallest region
# holding both (an axis joined in either is joined), which is their union for
# the nested regions a walk produces.  The walk of a first-iteration class
# (Section 3.5) starts at loop k with M holding every region of its body joined
# along it and the loops inside it.
# ---------------------------------------------------------------------------


@dataclass
class Stmt:
    kind: str            # 'kernel', 'copy-in' (X~ := X[slice]) or 'copy-out' (X[slice] := X~)
    regions: tuple       # Region records; a copy's are (source, target)


@dataclass
class Loop:
    index: str
    body: list           # Stmt and Loop nodes, in program order


def _temp(r: Region) -> Region:
    """The buffer X~ of a copied slice: the slice's kept axes, fixed by no loop."""
    kept = "".join(ch for ch, f in zip(r.letters, r.fixed) if not f)
    return Region(r.tensor + "~", kept, tuple(False for _ in kept))


def build_ast(variant):
    """The member's program: its loops, its copies at their levels, the kernel
    innermost.  Returns (root body, path to the kernel) where a path is a list
    of (body, position) from the root down."""
    ops = [Region(o.tensor, o.letters, o.fixed) for o in variant.operands]
    kernel_regions = tuple(_temp(r) if any(t == r.tensor for t, _ in variant.copies) else r for r in ops)
    kernel = Stmt("kernel", kernel_regions)
    by_level = {}
    for t, lv in variant.copies:
        by_level.setdefault(lv, []).append(t)
    reg = {r.tensor: r for r in ops}

    def body_at(level):
        """Statements of the body at loop position `level` (-1: the root)."""
        if level + 1 < len(variant.loops):
            inner = [Loop(variant.loops[level + 1], body_at(level + 1))]
        else:
            inner = [kernel]
        ins = [Stmt("copy-in", (reg[t], _temp(reg[t]))) for t in by_level.get(level, [])]
        outs = [Stmt("copy-out", (_temp(reg[t]), reg[t])) for t in by_level.get(level, []) if t == "C"]
        return ins + inner + outs

    root = body_at(-1)
    path, body = [], root
    while True:
        pos = next(i for i, n in enumerate(body) if isinstance(n, Loop) or n is kernel)
        path.append((body, pos))
        if body[pos] is kernel:
            return root, path
        body = body[pos].body


def _join(r: Region, loops) -> Region:
    return Region(r.tensor, r.letters, tuple(f and ch not in loops for ch, f in zip(r.letters, r.fixed)))


def _regions_of(node, joined):
    """Every region a node accesses, joined along `joined` and the loops inside it."""
    if isinstance(node, Stmt):
        return [_join(r, joined) for r in node.regions]
    out = []
    for n in node.body:
        out += _regions_of(n, set(joined) | {node.index})
    return out


def _tensors_of(node):
    return {r.tensor for r in _regions_of(node, set())}


def _merge(M: dict, regions):
    for r in regions:
        if r.tensor in M:
            q = M[r.tensor]
            M[r.tensor] = Region(r.tensor, r.letters, tuple(a and b for a, b in zip(q.fixed, r.fixed)))
        else:
            M[r.tensor] = r


def ast_distance(path, region: Region, extents: dict, start: int | None = None, root_gap: int = 0) -> int:
    """Access distance of ``region`` (accessed by the statement at the end of
    ``path``) by the walk above; ``start`` = loop depth of a first-iteration
    class (the walk then starts at that loop, M preloaded)."""
    M = {}
    op = region
    depth = len(path) - 1                 # path[depth] = (body, position) of the current node
    if start is not None:
        # path[start] holds the loop at depth `start` (the loop at loop position start)
        body, pos = path[start]
        loop = body[pos]
        inner = {loop.index} | {n.index for b, p in path[start + 1:] for n in [b[p]] if isinstance(n, Loop)}
        _merge(M, _regions_of(loop, set()))
        op = _join(op, inner)
        depth = start
    while True:
        body, pos = path[depth]
        for node in reversed(body[:pos]):                     # earlier statements, this iteration
            if op.tensor in _tensors_of(node):
                return sum(region_size(r, set(), extents) for r in M.values())
            _merge(M, _regions_of(node, set()))
        if depth == 0:                                        # case 3: the root
            return sum(region_size(r, set(), extents) for r in M.values()) + int(root_gap)
        pbody, ppos = path[depth - 1]
        loop = pbody[ppos]
        if not varies(op, loop.index, set()):                 # case 1: previous iteration of the loop
            for node in reversed(body[pos + 1:]):
                if op.tensor in _tensors_of(node):
                    break
                _merge(M, _regions_of(node, set()))
            return sum(region_size(r, set(), extents) for r in M.values())
        _merge(M, _regions_of(loop, set()))                   # case 2: the whole loop, joined along it
        op = _join(op, {loop.index})
        depth -= 1


def kernel_distances(variant, extents: dict, start: int | None = None, root_gaps: dict | None = None):
    """Access distances of the kernel's operands (copies' buffers for copied
    operands), keyed by the operand's tensor name ('A', 'B', 'C')."""
    root, path = build_ast(variant)
    body, pos = path[-1]
    out = {}
    for r in body[pos].regions:
        name = r.tensor.rstrip("~")
        gap = int((root_gaps or {}).get(name, 0))
        out[name] = ast_distance(path, r, extents, start=start, root_gap=gap)
    return out


def predict_member(variant, extents: dict, cache_elems: float, line_elems: int, stage: int = 5,
                   root_gaps: dict | None = None, keep_operand_only: bool = False):
    """predict_classes for the kernel of a family member, its operands and
    distances taken from the member's whole program (copies included): a
    copied operand is the copy's buffer, which no loop changes, so it is never
    prefetched and its setup access is the whole buffer."""
    root, path = build_ast(variant)
    body, pos = path[-1]
    ops = list(body[pos].regions)
    distance = lambda r, start, gap: ast_distance(path, r, extents, start=start, root_gap=gap)
    return predict_classes(ops, variant.loops, extents, cache_elems, line_elems, stage, root_gaps,
                           keep_operand_only, distance)
