"""GPU parity of batches: many contractions of the four batch patterns with
uneven extents in one graph launch, each against the oracle; graph replays
with new operands; tuning; error paths."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
tc = pytest.importorskip("paper_1409_8608_amd")
from paper_1409_8608_amd import workloads as wl  # noqa: E402


def _setup(dtype, integer, count=48, seed=5):
    import torch
    shapes, _ = wl.batch_shapes(count, seed=seed, cap_elems=1 << 18, free=(2, 90), con=(2, 24))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    plans, host, dev = [], [], []
    for item in shapes:
        A, B = wl.batch_values(item, integer=integer)
        p = tc.Plan(item["spec"], item["ext"], dtype)
        plans.append(p)
        host.append((A, B))
        dev.append((tc.to_device_fortran(A, tdt), tc.to_device_fortran(B, tdt),
                    tc.empty_fortran(p.shape("C"), tdt)))
    return shapes, plans, host, dev


def _check_all(shapes, host, Cs, dtype, exact, C0=None, alpha=None, beta=None):
    import torch
    torch.cuda.synchronize()
    for t, (item, (A, B), dC) in enumerate(zip(shapes, host, Cs)):
        Ar = A if dtype == "f64" else A.astype(np.float32).astype(np.float64)
        Br = B if dtype == "f64" else B.astype(np.float32).astype(np.float64)
        a = 1.0 if alpha is None else alpha[t]
        b = 0.0 if beta is None else beta[t]
        Cin = None if C0 is None else np.array(C0[t], order="F")
        ref = oracle.contract(item["spec"], item["ext"], Ar, Br, C=Cin, alpha=a, beta=b)
        got = dC.double().cpu().numpy()
        if exact:
            np.testing.assert_array_equal(got, ref, err_msg=f"member {t} {item['spec']} {item['ext']}")
        else:
            err = oracle.normwise_rel_err(got, ref)
            assert err <= (1e-12 if dtype == "f64" else 1e-5), (t, item, err)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_integer_exact_and_replay(dtype):
    import torch
    shapes, plans, host, dev = _setup(dtype, integer=True)
    batch = tc.Batch(plans)
    info = batch.info()
    assert info["members"] == len(plans) and info["tiles"] >= len(plans)
    As, Bs, Cs = zip(*dev)
    for C in Cs:
        C.fill_(float("nan"))
    batch.contract(As, Bs, Cs)
    _check_all(shapes, host, Cs, dtype, exact=True)
    # replay with new C buffers, alpha and beta
    Cs2 = [torch.full_like(C, 0.0) for C in Cs]
    rng = np.random.default_rng(1)
    C0 = [rng.integers(-2, 3, tuple(C.shape)).astype(np.float64) for C in Cs2]
    for C, c0 in zip(Cs2, C0):
        C.copy_(torch.from_numpy(c0))
    alphas = [float(rng.choice([1.0, -2.0, 0.5])) for _ in Cs2]
    betas = [float(rng.choice([0.0, 1.0, -1.0])) for _ in Cs2]
    batch.contract(As, Bs, Cs2, alphas, betas)
    batch.contract(As, Bs, Cs, [1.0] * len(Cs), [0.0] * len(Cs))     # third replay, first operands again
    _check_all(shapes, host, Cs2, dtype, exact=True, C0=C0, alpha=alphas, beta=betas)
    _check_all(shapes, host, Cs, dtype, exact=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_real_data_and_tune(dtype):
    shapes, plans, host, dev = _setup(dtype, integer=False, count=64, seed=9)
    batch = tc.Batch(plans)
    As, Bs, Cs = zip(*dev)
    batch.contract(As, Bs, Cs)
    _check_all(shapes, host, Cs, dtype, exact=False)
    batch.tune(2)
    assert batch.info()["tune_hit_rate"] == -1.0             # no score yet
    sc = batch.score(sample=16, seed=3)
    assert sc["n_sampled"] == 16 and sc["candidates_mean"] >= 3
    for q in ("seed", "topk", "tuned", "default"):
        assert 0.0 <= sc["argmin_" + q] <= sc["within5_" + q] <= 1.0
        assert sc["regret_" + q] >= 1.0
    assert batch.info()["tune_hit_rate"] == sc["within5_tuned"]
    # the tuning cache: a new batch of the same contractions starts from the kept choices
    again = tc.Batch(plans)
    assert [again.choice(t) for t in range(len(plans))] == [batch.choice(t) for t in range(len(plans))]
    for C in Cs:
        C.fill_(float("nan"))
    batch.contract(As, Bs, Cs)
    _check_all(shapes, host, Cs, dtype, exact=False)


def test_batch_errors():
    import torch
    p = tc.Plan("ab=ai,ib", dict(a=8, b=8, i=8), "f64")
    b = tc.Batch([p])
    x = torch.zeros(64, dtype=torch.float64, device="cuda").view(8, 8).t()
    y = torch.zeros(64, dtype=torch.float64, device="cuda").view(8, 8).t()
    c = torch.zeros(64, dtype=torch.float64, device="cuda").view(8, 8).t()
    with pytest.raises(tc.TcError) as e:
        b.contract([x], [y], [x], [1.0], [0.0])
    assert e.value.name == "TC_E_ALIAS"
    with pytest.raises(tc.TcError) as e:
        tc.tc_batch_tune(tc.Batch([p]).handle, 2)
    assert e.value.name == "TC_E_UNSUPPORTED"
    ps = tc.Plan("ab=ai,ib", dict(a=8, b=8, i=8), "f64", compute="fp8x3")
    with pytest.raises(tc.TcError) as e:
        tc.Batch([ps, p, ps])                # a split-FP8 plan's workspace serves one member
    assert e.value.name == "TC_E_UNSUPPORTED"
    with pytest.raises(tc.TcError) as e:
        tc.Batch([ps]).set_choice(0, tc.TC_VARIANT_FUSED, 0)   # no tile candidates
    assert e.value.name == "TC_E_VARIANT"
    pb = tc.Plan("ab=ai,ib", dict(a=8, b=8, i=8), "f64", compute="bf16x3")
    assert tc.Batch([pb, p, pb]).info()["members"] == 3   # split-BF16 tiles use no plan workspace


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_mixed_members(dtype):
    """Few and many summed positions, odd M, padded or permuted C, C's unit
    stride in B, a trace index, with alpha and beta, over two replays with new
    operands; integer data, exact."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    cases = [("abc=ai,ibc", dict(a=37, b=9, c=5, i=3), dict(C=[1, 40, 400])),
             ("abcd=ai,ibcd", dict(a=130, b=3, c=4, d=5, i=8), None),
             ("ba=ai,ib", dict(a=17, b=96, i=6), None),
             ("ab=ai,ibt", dict(a=64, b=33, i=5, t=2), None),
             ("abc=ai,ibc", dict(a=21, b=30, c=2, i=29), dict(A=[1, 24], C=[2 * 30, 2, 1])),
             ("abc=ija,jbic", dict(a=40, b=24, c=3, i=6, j=9), None),          # matrix core (K = 54)
             ("ab=iaj,jbi", dict(a=50, b=45, i=8, j=8), None)]                # matrix core (K = 64)
    rng = np.random.default_rng(17)
    plans = [tc.Plan(sp, ex, dtype, strides=st) for sp, ex, st in cases]
    batch = tc.Batch(plans)

    def views(sp, ex, st, arrays):
        out = []
        for name, x in zip("ABC", arrays):
            strides = (st or {}).get(name)
            if strides is None:
                out.append(tc.to_device_fortran(x, tdt))
                continue
            span = 1 + sum((n - 1) * s for n, s in zip(x.shape, strides))
            buf = torch.full((span,), float("nan"), dtype=tdt, device="cuda")
            v = torch.as_strided(buf, tuple(x.shape), tuple(strides))
            v.copy_(torch.from_numpy(np.ascontiguousarray(x)))
            out.append(v)
        return out
    for rep in range(2):
        host, dev = [], []
        for sp, ex, st in cases:
            A, B, C0 = wl.tensors(sp, ex, rng, integer=True, with_c=True)
            host.append((A, B, C0))
            dev.append(views(sp, ex, st, (A, B, C0)))
        alphas = [float(rng.choice([1.0, -2.0, 0.5])) for _ in cases]
        betas = [float(rng.choice([0.0, 1.0, -1.0])) for _ in cases]
        batch.contract([d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev], alphas, betas)
        torch.cuda.synchronize()
        for (sp, ex, st), (A, B, C0), d, al, be in zip(cases, host, dev, alphas, betas):
            ref = oracle.contract(sp, ex, A, B, C=np.array(C0, order="F"), alpha=al, beta=be)
            np.testing.assert_array_equal(d[2].double().cpu().numpy(), ref, err_msg=f"{sp} {ex} replay {rep}")
    info = batch.info()
    assert info["members"] == len(cases) and info["tiles"] >= len(cases)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_alpha_zero_reads_neither_input(dtype):
    """alpha = 0: C = beta * C without reading A or B (NaN-filled, or absent),
    beta = 0 without reading C either (NaN-filled); the other members of the
    same replay contract as usual."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    cases = [("abc=ai,ibc", dict(a=37, b=9, c=5, i=3)), ("ab=iaj,jbi", dict(a=50, b=45, i=8, j=8)),
             ("abc=ija,jbic", dict(a=40, b=24, c=3, i=6, j=9)), ("ab=ai,ib", dict(a=130, b=70, i=33))]
    plans = [tc.Plan(sp, ex, dtype) for sp, ex in cases]
    batch = tc.Batch(plans)
    rng = np.random.default_rng(23)
    host = [wl.tensors(sp, ex, rng, integer=True, with_c=True) for sp, ex in cases]
    alphas, betas = [0.0, 0.0, 2.0, 0.0], [-1.5, 0.0, -1.0, 1.0]
    As, Bs, Cs = [], [], []
    for (A, B, C0), p, al, be in zip(host, plans, alphas, betas):
        if al == 0.0:
            As.append(tc.empty_fortran(p.shape("A"), tdt).fill_(float("nan")))
            Bs.append(None if be == 1.0 else tc.empty_fortran(p.shape("B"), tdt).fill_(float("nan")))
        else:
            As.append(tc.to_device_fortran(A, tdt))
            Bs.append(tc.to_device_fortran(B, tdt))
        C = tc.to_device_fortran(C0, tdt)
        if be == 0.0:
            C.fill_(float("nan"))
        Cs.append(C)
    batch.contract(As, Bs, Cs, alphas, betas)
    torch.cuda.synchronize()
    for (sp, ex), (A, B, C0), C, al, be in zip(cases, host, Cs, alphas, betas):
        ref = oracle.contract(sp, ex, A, B, C=np.array(C0, order="F"), alpha=al, beta=be)
        np.testing.assert_array_equal(C.double().cpu().numpy(), ref, err_msg=f"{sp} alpha={al} beta={be}")


def _batch_candidates(plan):
    """The loop/kernel variants a batch member can run: the fused view and
    the gemm members whose loops are all free indices (no copies)."""
    sa, sb, sc = plan.letters
    contracted = [ch for ch in sa if ch in sb and ch not in sc]
    out = [tc.TC_VARIANT_FUSED]
    if len(contracted) == 1 and all(ch in sc for ch in set(sa + sb) - set(contracted)):
        out += [v["index"] for v in plan.variants()
                if v["kernel"] == "gemm" and not v["copies"] and not any(ch in contracted for ch in v["loops"])]
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_every_candidate_exact(dtype):
    """Every candidate of every member -- the fused view or a gemm member of
    the paper's family whose loops become batch dimensions, with each of the
    three tile shapes -- computes the contraction exactly on integer data
    inside the persistent kernel, alongside members running other candidates."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    cases = [("abc=ai,ibc", dict(a=37, b=9, c=5, i=3)), ("abcd=ai,ibcd", dict(a=20, b=3, c=4, d=5, i=7)),
             ("abc=ija,jbic", dict(a=40, b=24, c=3, i=6, j=9)), ("ab=iaj,jbi", dict(a=50, b=45, i=8, j=8)),
             ("abc=ai,ibc", dict(a=130, b=70, c=3, i=20))]
    plans = [tc.Plan(sp, ex, dtype) for sp, ex in cases]
    batch = tc.Batch(plans)
    rng = np.random.default_rng(29)
    host = [wl.tensors(sp, ex, rng, integer=True) for sp, ex in cases]
    As = [tc.to_device_fortran(A, tdt) for A, _, _ in host]
    Bs = [tc.to_device_fortran(B, tdt) for _, B, _ in host]
    Cs = [tc.empty_fortran(p.shape("C"), tdt) for p in plans]
    refs = [oracle.contract(sp, ex, A, B) for (sp, ex), (A, B, _) in zip(cases, host)]
    batch.contract(As, Bs, Cs)
    cands = [[(v, sh) for v in _batch_candidates(p) for sh in range(3)] for p in plans]
    assert [len(c) for c in cands] == [batch.choice(t)["candidates"] for t in range(len(plans))]
    assert [len(c) for c in cands] == [9, 21, 3, 3, 9]
    bound = batch.bind(As, Bs, Cs)
    for r in range(max(len(c) for c in cands)):
        for t, c in enumerate(cands):
            batch.set_choice(t, *c[(r + t) % len(c)])
        for C in Cs:
            C.fill_(float("nan"))
        batch.run(bound)
        torch.cuda.synchronize()
        for t, (C, ref) in enumerate(zip(Cs, refs)):
            np.testing.assert_array_equal(C.double().cpu().numpy(), ref,
                                          err_msg=f"{cases[t]} candidate {cands[t][(r + t) % len(cands[t])]}")
    with pytest.raises(tc.TcError) as e:
        batch.set_choice(2, 0, 0)                 # abc=ija,jbic has no member candidates
    assert e.value.name == "TC_E_VARIANT"


def test_batch_split_precision_members():
    """Split-precision members (BF16 and FP8 terms, FP64 and FP32 storage) in
    one graph with native members: integer data exact (single-term integers,
    exact partial sums); real data within the split forms' bounds against the
    oracle (split-BF16 tiles: componentwise within the FP32-accumulation bound
    of the oracle's exactly accumulated split result, and FP32 level against
    FP64); alpha = 0 with absent inputs; two replays with new operands."""
    import torch
    from gpu_util import split_bound
    from oracle import split as osplit
    cases = [("ab=iaj,jbi", dict(a=70, b=90, i=12, j=10), "f64", "bf16x3"),
             ("abc=ija,jbic", dict(a=40, b=33, c=7, i=5, j=11), "f32", "bf16x3"),
             ("abcd=ai,ibcd", dict(a=17, b=5, c=6, d=7, i=300), "f64", "fp8x3"),
             ("abc=ai,ibc", dict(a=37, b=9, c=5, i=3), "f64", "native"),
             ("ab=iaj,jbi", dict(a=50, b=45, i=8, j=8), "f64", "bf16x3")]
    plans = [tc.Plan(sp, ex, dt, compute=cm) for sp, ex, dt, cm in cases]
    batch = tc.Batch(plans)
    assert [batch.choice(t)["candidates"] for t in range(len(cases))] == [3, 3, 0, 9, 3]
    rng = np.random.default_rng(31)
    for rep, integer in enumerate((True, False)):
        host, dev = [], []
        for (sp, ex, dt, cm), p in zip(cases, plans):
            tdt = torch.float64 if dt == "f64" else torch.float32
            A, B, C0 = wl.tensors(sp, ex, rng, integer=integer, with_c=True)
            if dt == "f32":
                A, B, C0 = (x.astype(np.float32).astype(np.float64) for x in (A, B, C0))
            host.append((A, B, C0))
            dev.append([tc.to_device_fortran(A, tdt), tc.to_device_fortran(B, tdt), tc.to_device_fortran(C0, tdt)])
        alphas = [1.5, -2.0, 0.5, 1.0, 0.0]
        betas = [0.0, 1.0, -1.0, 0.5, 2.0]
        dev[4][0] = dev[4][1] = None                      # alpha = 0: A and B are not read
        batch.contract([d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev], alphas, betas)
        torch.cuda.synchronize()
        for t, ((sp, ex, dt, cm), (A, B, C0), d, al, be) in enumerate(zip(cases, host, dev, alphas, betas)):
            got = d[2].double().cpu().numpy()
            ref = oracle.contract(sp, ex, A, B, C=np.array(C0, order="F"), alpha=al, beta=be)
            if integer or al == 0.0 or cm == "native":
                if integer or al == 0.0:
                    np.testing.assert_array_equal(got, ref, err_msg=f"member {t} replay {rep}")
                else:
                    assert oracle.normwise_rel_err(got, ref) <= 1e-12
                continue
            absAB = oracle.contract(sp, ex, np.abs(A), np.abs(B))
            if cm == "bf16x3":
                sa_, sb_, sc_ = oracle.split_spec(sp)
                K = int(np.prod([ex[ch] for ch in sa_ if ch not in sc_]))
                ref_split = osplit.contract_split(sp, ex, A, B, C=np.array(C0, order="F"), alpha=al, beta=be)
                assert np.all(np.abs(got - ref_split) <= abs(al) * split_bound(K) * absAB
                              + 2.0 ** -50 * np.abs(ref_split)), (t, rep)
                assert oracle.normwise_rel_err(got, ref) <= 1e-5, (t, rep)
            else:                                         # FP8 terms: within 2^-9 |A||B|
                assert np.all(np.abs(got - ref) <= abs(al) * 2.0 ** -9 * absAB + 2.0 ** -50 * np.abs(ref)), (t, rep)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_bf16x3_tiles_wide_range(dtype):
    """Split-BF16 tiles on operands whose slices span many binades (FP64:
    per-slice scales 2^-300 .. 2^300, far outside BF16's and FP32's range, so
    only the per-row and per-column scaling keeps the terms representable;
    FP32: 2^-60 .. 2^60), every tile shape and both operand layouts, several
    K tiles and ragged edges: componentwise within the FP32-accumulation bound
    of the oracle's exactly accumulated split result (and, for FP32 storage,
    normwise at FP32 level)."""
    import torch
    from gpu_util import split_bound
    from oracle import split as osplit
    tdt = torch.float64 if dtype == "f64" else torch.float32
    span = 300 if dtype == "f64" else 60
    cases = [("ab=iaj,jbi", dict(a=130, b=70, i=7, j=9)),
             ("abc=ija,jbic", dict(a=33, b=20, c=3, i=6, j=5)),
             ("abc=ai,ibc", dict(a=150, b=17, c=4, i=37)),
             ("abcd=ai,ibcd", dict(a=40, b=9, c=3, d=2, i=20)),
             ("ba=ai,ib", dict(a=19, b=140, i=50))]
    rng = np.random.default_rng(77)
    plans, host, dev = [], [], []
    for sp, ex in cases:
        sa, sb, sc = oracle.split_spec(sp)
        A = np.array(rng.uniform(-1, 1, [ex[c] for c in sa]), order="F")
        B = np.array(rng.uniform(-1, 1, [ex[c] for c in sb]), order="F")
        for X, lets in ((A, sa), (B, sb)):
            shp = [X.shape[ax] if ch in sc else 1 for ax, ch in enumerate(lets)]
            X *= np.exp2(rng.integers(-span, span + 1, shp).astype(np.float64))
        if dtype == "f32":
            A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
        p = tc.Plan(sp, ex, dtype, compute="bf16x3")
        plans.append(p)
        host.append((A, B))
        dev.append((tc.to_device_fortran(A, tdt), tc.to_device_fortran(B, tdt), tc.empty_fortran(p.shape("C"), tdt)))
    batch = tc.Batch(plans)
    for shape in range(3):
        for t in range(len(cases)):
            batch.set_choice(t, tc.TC_VARIANT_FUSED, shape)
        for d in dev:
            d[2].fill_(float("nan"))
        batch.contract([d[0] for d in dev], [d[1] for d in dev], [d[2] for d in dev],
                       [1.0] * len(cases), [0.0] * len(cases))
        torch.cuda.synchronize()
        for t, ((sp, ex), (A, B), d) in enumerate(zip(cases, host, dev)):
            got = d[2].double().cpu().numpy()
            sa, sb, sc = oracle.split_spec(sp)
            K = int(np.prod([ex[c] for c in sa if c not in sc]))
            ref_split = osplit.contract_split(sp, ex, A, B)
            absAB = oracle.contract(sp, ex, np.abs(A), np.abs(B))
            # FP32 storage rounds the result once more
            tol = split_bound(K) * absAB + (2.0 ** -24 if dtype == "f32" else 2.0 ** -52) * np.abs(ref_split)
            assert np.all(np.abs(got - ref_split) <= tol), (sp, shape)
            if dtype == "f32":   # FP64 entries span 2^+-600: their squares overflow a norm
                assert oracle.normwise_rel_err(got, oracle.contract(sp, ex, A, B)) <= 1e-5, (sp, shape)
