"""GPU parity at the full workload sizes, in the configuration bench.py times,
on sampled outputs the oracle computes one slab at a time."""
import numpy as np
import pytest

import oracle
from oracle import split as sp
from gpu_util import split_bound, split_bound_fp8

pytestmark = pytest.mark.gpu
tc = pytest.importorskip("paper_1409_8608_amd")
from paper_1409_8608_amd import workloads as wl  # noqa: E402


def _dev(x, dtype):
    import torch
    return tc.to_device_fortran(x, torch.float64 if dtype == "f64" else torch.float32)


@pytest.mark.parametrize("n", [128, 640, 1024])
def test_smallk_cube_full_size(n):
    """C_abc = A_ai B_ibc, a=b=c=n, i=8, FP64, fused streaming kernel; four
    sampled c-slabs against the oracle."""
    import torch
    w = wl.smallk_cube(n, 8)
    p = tc.Plan(w["spec"], w["ext"], "f64")
    dA, dB = _dev(w["A"], "f64"), _dev(w["B"], "f64")
    dC = tc.empty_fortran(p.shape("C"), torch.float64)
    p.contract(dA, dB, dC)
    torch.cuda.synchronize()
    cs = np.sort(np.random.default_rng(n).choice(n, 4, replace=False))
    got = dC[:, :, torch.as_tensor(cs, device="cuda")].cpu().numpy()
    ref = oracle.contract("abc=ai,ibc", dict(a=n, b=n, c=len(cs), i=8), w["A"], np.asfortranarray(w["B"][:, :, cs]))
    assert oracle.normwise_rel_err(got, ref) <= 1e-12
    assert np.isfinite(dC.sum().item())


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_permuted_full_size(dtype):
    """C_abc = A_ija B_jbic, 256^3 x 32^2, fused matrix-core kernel; two c-slabs."""
    import torch
    w = wl.permuted(256, 32)
    p = tc.Plan(w["spec"], w["ext"], dtype)
    dA, dB = _dev(w["A"], dtype), _dev(w["B"], dtype)
    dC = tc.empty_fortran(p.shape("C"), torch.float64 if dtype == "f64" else torch.float32)
    p.contract(dA, dB, dC)
    torch.cuda.synchronize()
    cs = np.array([3, 200])
    got = dC[:, :, torch.as_tensor(cs, device="cuda")].double().cpu().numpy()
    A = w["A"] if dtype == "f64" else w["A"].astype(np.float32).astype(np.float64)
    B = w["B"] if dtype == "f64" else w["B"].astype(np.float32).astype(np.float64)
    ref = oracle.contract(w["spec"], dict(w["ext"], c=len(cs)), A, np.asfortranarray(B[:, :, :, cs]))
    assert oracle.normwise_rel_err(got, ref) <= (1e-12 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("compute", ["native", "bf16x3", "fp8x3"])
def test_scaled_matrix_full_size(compute):
    """C_ab = A_iaj B_jbi, a=b=4096, i=j=64 with per-slice scales: FP64 plain,
    split-BF16 and split-FP8 on sampled rows and columns; the split forms also
    within their bounds of the exactly accumulated split oracle."""
    import torch
    w = wl.scaled_matrix(4096, 64)
    p = tc.Plan(w["spec"], w["ext"], "f64", compute=compute)
    dA, dB = _dev(w["A"], "f64"), _dev(w["B"], "f64")
    dC = tc.empty_fortran(p.shape("C"), torch.float64)
    p.contract(dA, dB, dC)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(4096, 16, replace=False))
    cols = np.sort(rng.choice(4096, 16, replace=False))
    got = dC[torch.as_tensor(rows, device="cuda")][:, torch.as_tensor(cols, device="cuda")].cpu().numpy()
    As, Bs = np.asfortranarray(w["A"][:, rows, :]), np.asfortranarray(w["B"][:, cols, :])
    ext_s = dict(a=len(rows), b=len(cols), i=64, j=64)
    ref = oracle.contract(w["spec"], ext_s, As, Bs)
    if compute == "native":
        assert oracle.normwise_rel_err(got, ref) <= 1e-12
    else:
        kind = "bf16" if compute == "bf16x3" else "fp8"
        absAB = oracle.contract(w["spec"], ext_s, np.abs(As), np.abs(Bs))
        # slices are per free index, so sampling rows and columns keeps them
        ref_split = sp.contract_split(w["spec"], ext_s, As, Bs, kind=kind)
        bound = split_bound(64 * 64) if kind == "bf16" else split_bound_fp8(64 * 64)
        assert np.all(np.abs(got - ref_split) <= bound * absAB)
        if kind == "bf16":
            assert oracle.normwise_rel_err(got, ref) <= 1e-5
        else:
            assert np.all(np.abs(got - ref) <= 2.0 ** -9 * absAB)


def test_batch_full_size_sampled():
    """All 4096 batch members in one graph replay (FP32), 12 members checked."""
    import torch
    shapes, _ = wl.batch_shapes(4096)
    plans, As, Bs, Cs = [], [], [], []
    gen = torch.Generator(device="cuda")
    gen.manual_seed(51)
    for it in shapes:
        p = tc.Plan(it["spec"], it["ext"], "f32")
        plans.append(p)
        As.append(tc.empty_fortran(p.shape("A"), torch.float32).uniform_(-1, 1, generator=gen))
        Bs.append(tc.empty_fortran(p.shape("B"), torch.float32).uniform_(-1, 1, generator=gen))
        Cs.append(tc.empty_fortran(p.shape("C"), torch.float32).fill_(float("nan")))
    b = tc.Batch(plans)
    b.contract(As, Bs, Cs)
    torch.cuda.synchronize()
    for t in np.random.default_rng(2).choice(4096, 12, replace=False):
        it = shapes[t]
        ref = oracle.contract(it["spec"], it["ext"], As[t].double().cpu().numpy(), Bs[t].double().cpu().numpy())
        assert oracle.normwise_rel_err(Cs[t].double().cpu().numpy(), ref) <= 1e-5, (t, it)
    # every member was written (no NaN left from the fill)
    assert all(bool(torch.isfinite(C).all()) for C in Cs)


def test_case_study_members_at_sweep_size():
    """All 36 members of C_abc = A_ai B_ibc at a=b=c=128, i=8 (the sweep's
    first size), each on two sampled c-slabs."""
    import torch
    w = wl.smallk_cube(128, 8)
    p = tc.Plan(w["spec"], w["ext"], "f64")
    dA, dB = _dev(w["A"], "f64"), _dev(w["B"], "f64")
    dC = tc.empty_fortran(p.shape("C"), torch.float64)
    cs = np.array([5, 77])
    ref = oracle.contract("abc=ai,ibc", dict(a=128, b=128, c=2, i=8), w["A"], np.asfortranarray(w["B"][:, :, cs]))
    for v in range(36):
        p.set_variant(v)
        dC.fill_(float("nan"))
        p.contract(dA, dB, dC)
        torch.cuda.synchronize()
        got = dC[:, :, torch.as_tensor(cs, device="cuda")].cpu().numpy()
        assert oracle.normwise_rel_err(got, ref) <= 1e-12, v


def test_permuted_gemm_members_full_size():
    """The eight copy+gemm members of Test 3 at 256^3 x 32^2 (FP64)."""
    import torch
    w = wl.permuted(256, 32)
    p = tc.Plan(w["spec"], w["ext"], "f64")
    dA, dB = _dev(w["A"], "f64"), _dev(w["B"], "f64")
    dC = tc.empty_fortran(p.shape("C"), torch.float64)
    cs = np.array([7])
    ref = oracle.contract(w["spec"], dict(w["ext"], c=1), w["A"], np.asfortranarray(w["B"][:, :, :, cs]))
    for v in range(168, 176):
        p.set_variant(v)
        dC.fill_(float("nan"))
        p.contract(dA, dB, dC)
        torch.cuda.synchronize()
        got = dC[:, :, torch.as_tensor(cs, device="cuda")].cpu().numpy()
        assert oracle.normwise_rel_err(got, ref) <= 1e-12, p.variants()[v]["name"]
