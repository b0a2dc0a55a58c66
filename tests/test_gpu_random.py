"""Seeded random contractions on the GPU against the oracle: random index
classes (free, contracted, batch, trace), extents, storage orders (Fortran,
permuted axes, padded strides), storage types, alpha and beta, through the
fused path.  Each case prints its seed and spec before it runs."""
import numpy as np
import pytest

from gpu_util import check

pytestmark = pytest.mark.gpu
tc = pytest.importorskip("paper_1409_8608_amd")


def _draw_case(seed):
    rng = np.random.default_rng(1000 + seed)
    letters = list("abcdefgijklmst")
    rng.shuffle(letters)
    n = dict(fa=int(rng.integers(0, 3)), fb=int(rng.integers(0, 3)), k=int(rng.integers(0, 4)),
             bt=int(rng.random() < 0.3), ta=int(rng.random() < 0.2), tb=int(rng.random() < 0.2))
    if n["fa"] + n["fb"] + n["bt"] == 0:
        n["fa"] = 1
    groups, at = {}, 0
    for key in ("fa", "fb", "k", "bt", "ta", "tb"):
        groups[key] = letters[at:at + n[key]]
        at += n[key]
    perm = lambda xs: "".join(rng.permutation(xs)) if xs else ""
    sa = perm(groups["fa"] + groups["k"] + groups["bt"] + groups["ta"])
    sb = perm(groups["fb"] + groups["k"] + groups["bt"] + groups["tb"])
    sc = perm(groups["fa"] + groups["fb"] + groups["bt"])
    spec = f"{sc}={sa},{sb}"
    ext = {ch: int(np.exp(rng.uniform(0, np.log(48)))) for ch in set(sa + sb + sc)}

    def size(s):
        return int(np.prod([ext[ch] for ch in s])) if s else 1
    # operands up to 2^18 elements, contraction length up to 2^13
    K = "".join(groups["k"] + groups["ta"] + groups["tb"])
    while max(size(sa), size(sb), size(sc)) > (1 << 18) or size(K) > (1 << 13):
        big = max(ext, key=ext.get)
        ext[big] = max(1, ext[big] // 2)
    dtype = "f64" if rng.random() < 0.6 else "f32"
    alpha = float(rng.choice([1.0, -0.5, 2.0]))
    beta = float(rng.choice([0.0, 0.0, 1.0, -1.5]))
    return rng, spec, ext, dtype, alpha, beta


def _layout(shape, rng):
    """Strides of a permuted, possibly padded storage order (one-to-one)."""
    nd = len(shape)
    order = list(rng.permutation(nd)) if rng.random() < 0.5 else list(range(nd))
    strides, run = [0] * nd, 1
    for ax in order:
        strides[ax] = run
        run *= shape[ax] + (1 if rng.random() < 0.3 else 0)
    span = 1 + sum((e - 1) * s for e, s in zip(shape, strides)) if nd else 1
    return strides, span


@pytest.mark.parametrize("seed", range(160))
def test_random_contraction(seed):
    import torch
    from paper_1409_8608_amd import workloads as wl
    rng, spec, ext, dtype, alpha, beta = _draw_case(seed)
    print(f"case seed={seed} spec={spec} ext={ext} dtype={dtype} alpha={alpha} beta={beta}", flush=True)
    A, B, C0 = wl.tensors(spec, ext, rng, "normal", with_c=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    views, strides = [], {}
    for name, x in (("A", A), ("B", B), ("C", C0)):
        st, span = _layout(list(x.shape), rng)
        buf = torch.full((span + 8,), float("nan"), dtype=tdt, device="cuda")
        v = torch.as_strided(buf, tuple(x.shape), tuple(st))
        v.copy_(torch.from_numpy(np.array(x, order="C")))   # keeps 0-d operands 0-d
        views.append(v)
        strides[name] = st
    p = tc.Plan(spec, ext, dtype, strides=strides)
    p.contract(views[0], views[1], views[2], alpha, beta)
    torch.cuda.synchronize()
    got = views[2].double().cpu().numpy()
    check(spec, ext, A, B, got, dtype, C0=C0, alpha=alpha, beta=beta)


def _draw_family_case(seed):
    """Paper index classes only (free and contracted), at most 4 indices per
    operand, small extents so that every member runs quickly."""
    rng = np.random.default_rng(5000 + seed)
    letters = list("abcdijkl")
    rng.shuffle(letters)
    nfa, nfb, nk = int(rng.integers(0, 3)), int(rng.integers(0, 3)), int(rng.integers(1, 3))
    if nfa + nfb == 0:
        nfa = 1
    fa, fb, k = letters[:nfa], letters[nfa:nfa + nfb], letters[nfa + nfb:nfa + nfb + nk]
    perm = lambda xs: "".join(rng.permutation(xs)) if xs else ""
    sa, sb, sc = perm(fa + k), perm(fb + k), perm(fa + fb)
    ext = {ch: int(rng.integers(1, 20)) for ch in set(sa + sb + sc)}
    dtype = "f64" if rng.random() < 0.6 else "f32"
    return rng, f"{sc}={sa},{sb}", ext, dtype


@pytest.mark.parametrize("seed", range(40))
def test_random_family_members(seed):
    import torch
    from paper_1409_8608_amd import workloads as wl
    rng, spec, ext, dtype = _draw_family_case(seed)
    A, B, C0 = wl.tensors(spec, ext, rng, "normal", with_c=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    views, strides = [], {}
    for name, x in (("A", A), ("B", B), ("C", C0)):
        st, span = _layout(list(x.shape), rng)
        buf = torch.full((span + 8,), float("nan"), dtype=tdt, device="cuda")
        v = torch.as_strided(buf, tuple(x.shape), tuple(st))
        v.copy_(torch.from_numpy(np.array(x, order="C")))
        views.append(v)
        strides[name] = st
    p = tc.Plan(spec, ext, dtype, strides=strides)
    infos = p.variants()
    picks = rng.choice(len(infos), min(8, len(infos)), replace=False)
    for v in sorted(int(x) for x in picks):
        print(f"case seed={seed} spec={spec} ext={ext} dtype={dtype} member={infos[v]['name']}", flush=True)
        p.set_variant(v)
        views[2].copy_(torch.from_numpy(np.array(C0, order="C")))
        if not infos[v]["runs_on_gpu"]:
            with pytest.raises(tc.TcError) as e:
                p.contract(views[0], views[1], views[2], 1.5, -1.0)
            assert e.value.name == "TC_E_UNSUPPORTED"
            continue
        p.contract(views[0], views[1], views[2], 1.5, -1.0)
        torch.cuda.synchronize()
        check(spec, ext, A, B, views[2].double().cpu().numpy(), dtype, C0=C0, alpha=1.5, beta=-1.0)


@pytest.mark.parametrize("seed", range(60))
def test_random_complex_contraction(seed):
    """The same random cases in complex storage (both types), complex alpha and
    beta, against the complex oracle."""
    import torch
    import oracle
    from paper_1409_8608_amd import workloads as wl
    rng, spec, ext, dtype, alpha, beta = _draw_case(seed)
    dtype = "c128" if dtype == "f64" else "c64"
    alpha = complex(alpha, float(rng.choice([0.0, 0.5, -1.0])))
    beta = complex(beta, float(rng.choice([0.0, 0.0, 0.25])))
    print(f"case seed={seed} spec={spec} ext={ext} dtype={dtype} alpha={alpha} beta={beta}", flush=True)
    A, B = wl.complex_tensors(spec, ext, rng)
    sc = spec.split("=")[0]
    shape_c = [ext[ch] for ch in sc]
    C0 = np.array(rng.uniform(-1, 1, size=shape_c) + 1j * rng.uniform(-1, 1, size=shape_c), dtype=np.complex128,
                  order="F")
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    views, strides = [], {}
    for name, x in (("A", A), ("B", B), ("C", C0)):
        st, span = _layout(list(x.shape), rng)
        buf = torch.full((span + 8,), complex(np.nan, np.nan), dtype=tdt, device="cuda")
        v = torch.as_strided(buf, tuple(x.shape), tuple(st))
        v.copy_(torch.from_numpy(np.array(x, order="C")))
        views.append(v)
        strides[name] = st
    p = tc.Plan(spec, ext, dtype, strides=strides)
    p.contract(views[0], views[1], views[2], alpha, beta)
    torch.cuda.synchronize()
    got = np.array(views[2].cpu().numpy(), dtype=np.complex128)

    def rnd(x):
        return np.array(x if dtype == "c128" else x.astype(np.complex64), dtype=np.complex128, order="F")
    ref = oracle.contract(spec, ext, rnd(A), rnd(B), C=rnd(C0), alpha=alpha, beta=beta)
    err = oracle.normwise_rel_err(got, ref)
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert err <= tol, f"normwise error {err:.3e} > {tol:.1e}"
