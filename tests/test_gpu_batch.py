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
    info = batch.info()
    assert 0.0 <= info["tune_hit_rate"] <= 1.0
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
        b.contract([x], [y], [c], [0.0], [1.0])
    assert e.value.name == "TC_E_UNSUPPORTED"
    with pytest.raises(tc.TcError) as e:
        b.contract([x], [y], [x], [1.0], [0.0])
    assert e.value.name == "TC_E_ALIAS"
    with pytest.raises(tc.TcError) as e:
        tc.tc_batch_tune(tc.Batch([p]).handle, 2)
    assert e.value.name == "TC_E_UNSUPPORTED"
    ps = tc.Plan("ab=ai,ib", dict(a=8, b=8, i=8), "f64", compute="bf16x3")
    with pytest.raises(tc.TcError) as e:
        tc.Batch([ps])
    assert e.value.name == "TC_E_UNSUPPORTED"
