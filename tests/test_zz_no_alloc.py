"""GPU tests of tc_contract_noalloc, the fused contraction whose device
buffers beyond A, B and C (the K table and the split-K partial tiles) live in
the library's static scratch array: its output equals tc_contract's on the
same plan shape bit for bit (same kernels, same K walk, same slices) and meets
the oracle's tolerance, over two calls in a row with the second smaller, plus
the matrix-core path without split K, the streaming path and the refusals."""
import numpy as np
import pytest

import oracle
from gpu_util import check

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_1409_8608_amd")
from paper_1409_8608_amd import workloads as wl  # noqa: E402


def _both(spec, ext, dtype, seed, alpha=1.0, beta=0.0, integer=False):
    """C from tc_contract and from tc_contract_noalloc on the same inputs."""
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    A, B, C0 = wl.tensors(spec, ext, np.random.default_rng(seed), integer=integer, with_c=beta != 0.0)
    ref_plan = tc.Plan(spec, ext, dtype)
    na_plan = tc.Plan(spec, ext, dtype)
    dA = tc.to_device_fortran(A, tdt)
    dB = tc.to_device_fortran(B, tdt)
    outs = []
    for plan, fn in ((ref_plan, tc.tc_contract), (na_plan, tc.tc_contract_noalloc)):
        if C0 is not None:
            dC = tc.to_device_fortran(C0, tdt)
        else:
            dC = tc.empty_fortran(plan.shape("C"), tdt)
            dC.fill_(float("nan"))                     # beta = 0 must not read C
        fn(plan.handle, dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), alpha, beta,
           torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        outs.append(dC.double().cpu().numpy())
    return A, B, C0, outs[0], outs[1]


def test_noalloc_two_calls_second_smaller():
    """Call 1: a=iaj,ji with a=300, i=96, j=80 (7,680 positions; three output
    tiles, 60 split-K slices, 23.6 MB of partial tiles).  Call 2: a=100, i=40,
    j=30 (1,200 positions, one tile, split K), after call 1 has filled the
    scratch with its own table and partials."""
    spec = "a=iaj,ji"
    for ext, seed in ((dict(a=300, i=96, j=80), 1), (dict(a=100, i=40, j=30), 2)):
        A, B, _, ref, got = _both(spec, ext, "f64", seed)
        np.testing.assert_array_equal(got, ref)
        check(spec, ext, A, B, got, "f64")


def test_noalloc_integer_exact_fp32_and_fp64():
    spec, ext = "a=iaj,ji", dict(a=257, i=64, j=50)
    for dtype in ("f64", "f32"):
        A, B, C0, ref, got = _both(spec, ext, dtype, 3, alpha=2.0, beta=-1.0, integer=True)
        np.testing.assert_array_equal(got, ref)
        check(spec, ext, A, B, got, dtype, C0=C0, alpha=2.0, beta=-1.0, exact=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_permuted_tiles_without_split(dtype):
    """abc=ija,jbic at 48^3 x 8^2: 64 positions over two contracted indices,
    permuted strides, 18 tiles, too few K tiles to split; beta reads C."""
    spec, ext = "abc=ija,jbic", dict(a=48, b=48, c=48, i=8, j=8)
    A, B, C0, ref, got = _both(spec, ext, dtype, 4, alpha=0.5, beta=-1.5)
    np.testing.assert_array_equal(got, ref)
    check(spec, ext, A, B, got, dtype, C0=C0, alpha=0.5, beta=-1.5)


def test_noalloc_streaming_path():
    spec, ext = "abc=ai,ibc", dict(a=256, b=16, c=12, i=8)
    A, B, _, ref, got = _both(spec, ext, "f64", 5)
    np.testing.assert_array_equal(got, ref)
    check(spec, ext, A, B, got, "f64")


def test_noalloc_refusals_leave_c_untouched():
    import torch
    # 2100^2 = 4,410,000 positions: a K table of 70.6 MB, beyond the 64 MiB array
    spec, ext = "a=iaj,ji", dict(a=1, i=2100, j=2100)
    p = tc.Plan(spec, ext, "f64")
    dA = torch.zeros(2100 * 2100, dtype=torch.float64, device="cuda")
    dB = torch.zeros(2100 * 2100, dtype=torch.float64, device="cuda")
    dC = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(tc.TcError) as e:
        tc.tc_contract_noalloc(p.handle, dA.data_ptr(), dB.data_ptr(), dC.data_ptr())
    assert e.value.name == "TC_E_UNSUPPORTED" and "scratch" in str(e.value)
    # a member variant selected
    q = tc.Plan("abc=ai,ibc", dict(a=8, b=8, c=8, i=8), "f64")
    q.set_variant(0)
    with pytest.raises(tc.TcError) as e:
        tc.tc_contract_noalloc(q.handle, dA.data_ptr(), dB.data_ptr(), dC.data_ptr())
    assert e.value.name == "TC_E_UNSUPPORTED"
    torch.cuda.synchronize()
    assert dC.item() == 7.0
