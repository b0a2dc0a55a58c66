"""GPU parity: the fused kernels and every family member against the FP64
oracle, through the C ABI.  Tolerances: FP64 normwise <= 1e-12, FP32 <= 1e-5
(against the oracle on the FP32-rounded inputs); integer data bit-exact."""
import numpy as np
import pytest

import oracle
from gpu_util import check, run

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_1409_8608_amd")
from paper_1409_8608_amd import workloads as wl  # noqa: E402


def _plan(spec, ext, dtype="f64", strides=None, compute="native"):
    return tc.Plan(spec, ext, dtype=dtype, strides=strides, compute=compute)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_smallk_cube(dtype):
    w = wl.smallk_cube(64, 8)
    p = _plan(w["spec"], w["ext"], dtype)
    got = run(p, w["A"], w["B"], dtype=dtype)
    check(w["spec"], w["ext"], w["A"], w["B"], got, dtype)


def test_fused_smallk_integer_exact_and_beta():
    w = wl.smallk_cube(64, 8, integer=True, with_c=True)
    p = _plan(w["spec"], w["ext"])
    got = run(p, w["A"], w["B"], w["C"], alpha=2.0, beta=-0.5)
    check(w["spec"], w["ext"], w["A"], w["B"], got, C0=w["C"], alpha=2.0, beta=-0.5, exact=True)


# Streaming shapes: M a whole number of wave spans (128 doubles, 256 floats),
# M with a tail for the general kernel, N of two dimensions that do not merge,
# K padded up to the kernel's template size (1, 5, 12), K = 32, odd M (no
# vector path at all), N not a whole number of block column sets.  Beyond 8
# summed positions only M in whole wave spans streams, beyond 16 nothing does
# (matrix cores).
STREAM_SHAPES = [
    ("abc=ai,ibc", dict(a=384, b=7, c=5, i=8)),
    ("abc=ai,ibc", dict(a=300, b=9, c=4, i=5)),
    ("abc=ai,icb", dict(a=256, b=6, c=7, i=12)),
    ("abc=ai,ibc", dict(a=256, b=3, c=11, i=32)),
    ("ab=ai,ib", dict(a=1024, b=33, i=1)),
    ("abc=ai,ibc", dict(a=129, b=5, c=3, i=7)),
    ("abc=aij,jibc", dict(a=512, b=3, c=5, i=3, j=4)),
    ("abc=aij,jibc", dict(a=520, b=3, c=5, i=3, j=4)),           # 12 positions, ragged M: matrix cores
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("K", [12, 16])
def test_fused_stream_general_kernel_misaligned(dtype, K):
    """M in whole wave spans but A starting one element into its allocation:
    the wave kernel needs 16-byte rows, so the general streaming kernel (9..16
    positions) covers all of M."""
    import torch
    spec, ext = "abc=ai,ibc", dict(a=256, b=5, c=7, i=K)
    A, B, C0 = wl.tensors(spec, ext, np.random.default_rng(9), integer=True, with_c=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p = _plan(spec, ext, dtype)
    store = torch.zeros(1 + 256 * K, dtype=tdt, device="cuda")
    dA = torch.as_strided(store, (256, K), (1, 256), 1)
    dA.copy_(torch.from_numpy(A))
    dB = tc.to_device_fortran(B, tdt)
    dC = tc.to_device_fortran(C0, tdt)
    p.contract(dA, dB, dC, 2.0, -1.0)
    torch.cuda.synchronize()
    check(spec, ext, A, B, dC.double().cpu().numpy(), dtype, C0=C0, alpha=2.0, beta=-1.0, exact=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", STREAM_SHAPES)
def test_fused_stream_shapes(dtype, spec, ext):
    rng = np.random.default_rng(7)
    A, B, C0 = wl.tensors(spec, ext, rng, "normal", with_c=True)
    p = _plan(spec, ext, dtype)
    got = run(p, A, B, dtype=dtype)
    check(spec, ext, A, B, got, dtype)
    got = run(p, A, B, C0, alpha=-1.5, beta=0.25, dtype=dtype)
    check(spec, ext, A, B, got, dtype, C0=C0, alpha=-1.5, beta=0.25)


@pytest.mark.parametrize("spec,ext", STREAM_SHAPES[:5])
def test_fused_stream_integer_exact(spec, ext):
    A, B, C0 = wl.tensors(spec, ext, np.random.default_rng(8), integer=True, with_c=True)
    for dtype in ("f64", "f32"):
        p = _plan(spec, ext, dtype)
        got = run(p, A, B, dtype=dtype)
        check(spec, ext, A, B, got, dtype, exact=True)
        got = run(p, A, B, C0, alpha=2.0, beta=-1.0, dtype=dtype)
        check(spec, ext, A, B, got, dtype, C0=C0, alpha=2.0, beta=-1.0, exact=True)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", [
    ("abc=ija,jbic", dict(a=40, b=33, c=7, i=5, j=11)),          # ragged tiles, permuted strides
    ("ab=iaj,jbi", dict(a=130, b=70, i=9, j=6)),
    ("abcd=ai,ibcd", dict(a=17, b=5, c=6, d=7, i=40)),            # K > 32: matrix cores
    ("abc=ai,ibc", dict(a=200, b=9, c=3, i=100)),
    ("ab=ai,ib", dict(a=129, b=257, i=64)),
    ("abc=bi,iac", dict(a=64, b=48, c=5, i=33)),                   # C's unit index comes from B
])
def test_fused_mfma_shapes(dtype, spec, ext):
    rng = np.random.default_rng(3)
    A, B, _ = wl.tensors(spec, ext, rng, "normal")
    p = _plan(spec, ext, dtype)
    got = run(p, A, B, dtype=dtype)
    check(spec, ext, A, B, got, dtype)


# Operand staging modes of the matrix-core kernel: 16-byte K chunks where the
# K table's chunks are contiguous and every row offset is a chunk multiple,
# single elements otherwise.  Ragged M/N tiles, K padded inside a tile (i=20),
# a K extent that splits a chunk (i=22: element loads), a row stride that is a
# multiple of 2 but not 4 (FP64 chunks, FP32 elements), two contracted indices.
MFMA_CHUNK_SHAPES = [
    ("abc=ija,jbic", dict(a=40, b=36, c=7, i=8, j=12)),
    ("ab=ia,ib", dict(a=100, b=50, i=20)),
    ("ab=ia,ib", dict(a=64, b=70, i=22)),
    ("ab=ia,ib", dict(a=90, b=33, i=18)),
    ("ab=iaj,jbi", dict(a=130, b=70, i=8, j=8)),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", MFMA_CHUNK_SHAPES)
def test_fused_mfma_chunk_loads(dtype, spec, ext):
    rng = np.random.default_rng(13)
    A, B, C0 = wl.tensors(spec, ext, rng, "normal", with_c=True)
    p = _plan(spec, ext, dtype)
    got = run(p, A, B, dtype=dtype)
    check(spec, ext, A, B, got, dtype)
    got = run(p, A, B, C0, alpha=0.5, beta=-2.0, dtype=dtype)
    check(spec, ext, A, B, got, dtype, C0=C0, alpha=0.5, beta=-2.0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fused_mfma_unaligned_base(dtype):
    """Operands that start one element past a 16-byte boundary take the
    element loads; same result as the aligned call."""
    torch = pytest.importorskip("torch")
    spec, ext = "ab=ia,ib", dict(a=100, b=50, i=20)
    A, B, _ = wl.tensors(spec, ext, np.random.default_rng(14), "normal")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p = _plan(spec, ext, dtype)
    bufA = torch.zeros(A.size + 1, dtype=tdt, device="cuda")
    bufB = torch.zeros(B.size + 1, dtype=tdt, device="cuda")
    dA = torch.as_strided(bufA, A.shape, (1, A.shape[0]), 1)
    dB = torch.as_strided(bufB, B.shape, (1, B.shape[0]), 1)
    dA.copy_(torch.from_numpy(A))
    dB.copy_(torch.from_numpy(B))
    dC = tc.empty_fortran(p.shape("C"), tdt).fill_(float("nan"))
    p.contract(dA, dB, dC)
    torch.cuda.synchronize()
    check(spec, ext, A, B, dC.double().cpu().numpy(), dtype)


# Split K: few output tiles and a long contraction (the paper's Test 2,
# C_a = A_iaj B_ji, and a small matrix product with K in the thousands): the
# fused kernel splits K over blocks and sums the slices in a fixed order.
# K values not a multiple of 16 leave padding in the last tile.
SPLITK_SHAPES = [
    ("a=iaj,ji", dict(a=100, i=120, j=90)),
    ("ab=ia,ib", dict(a=150, b=130, i=5000)),
    ("a=iaj,ji", dict(a=300, i=64, j=201)),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", SPLITK_SHAPES)
def test_fused_split_k(dtype, spec, ext):
    rng = np.random.default_rng(17)
    A, B, C0 = wl.tensors(spec, ext, rng, "normal", with_c=True)
    p = _plan(spec, ext, dtype)
    got = run(p, A, B, dtype=dtype)
    check(spec, ext, A, B, got, dtype)
    got = run(p, A, B, C0, alpha=0.5, beta=-1.5, dtype=dtype)
    check(spec, ext, A, B, got, dtype, C0=C0, alpha=0.5, beta=-1.5)


def test_split_k_workspace_is_reported():
    """The split-K partial tiles are part of the plan's workspace: the Test 2
    shape a=100, i=120, j=90 (one output tile, 675 K tiles) uses slices of
    9 K tiles, 75 x 128 x 128 doubles."""
    spec, ext = "a=iaj,ji", dict(a=100, i=120, j=90)
    p = _plan(spec, ext)
    p.prepare()
    ktab = 2 * 8 * 10800                 # (A, B) offset pairs of the K table
    assert tc.tc_plan_workspace(p.handle) >= ktab + 75 * 128 * 128 * 8


def test_fused_split_k_integer_exact():
    spec, ext = "a=iaj,ji", dict(a=100, i=120, j=90)
    A, B, C = wl.tensors(spec, ext, np.random.default_rng(21), integer=True, with_c=True)
    for dtype in ("f64", "f32"):
        p = _plan(spec, ext, dtype)
        got = run(p, A, B, C, alpha=1.0, beta=-1.0, dtype=dtype)
        check(spec, ext, A, B, got, dtype, C0=C, alpha=1.0, beta=-1.0, exact=True)


# Family members with long kernels and few outputs (the paper's Test 2): the
# member body gives each output 8 lanes (length 40) or 64 lanes (length 130).
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [40, 130])
def test_test2_members_long_kernels(dtype, n):
    import torch
    spec, ext = "a=iaj,ji", dict(a=n, i=n, j=17)
    rng = np.random.default_rng(n)
    A, B, C0 = wl.tensors(spec, ext, rng, "normal", with_c=True)
    p = _plan(spec, ext, dtype)
    assert len(p.variants()) == 8
    for v in range(8):
        p.set_variant(v)
        got = run(p, A, B, C0, alpha=2.0, beta=0.5, dtype=dtype)
        check(spec, ext, A, B, got, dtype, C0=C0, alpha=2.0, beta=0.5)


def test_test2_members_integer_exact():
    spec, ext = "a=iaj,ji", dict(a=130, i=130, j=9)
    A, B, C = wl.tensors(spec, ext, np.random.default_rng(23), integer=True, with_c=True)
    p = _plan(spec, ext)
    for v in range(8):
        p.set_variant(v)
        got = run(p, A, B, C, alpha=1.0, beta=2.0)
        check(spec, ext, A, B, got, C0=C, alpha=1.0, beta=2.0, exact=True)


# Index classes outside the paper's definition, on the fused kernel: batch
# indices (in A, B and C) become the matrix-core kernel's batch dimensions,
# trace indices (one input only) contracted dimensions with stride 0 in the
# other input.  K <= 32 with a trace index of B and no batch index runs the
# streaming kernel; the Hadamard form bc=tbc,sbc has one output per tile.
GENERAL_SHAPES = [
    ("abc=aic,ibc", dict(a=70, b=40, c=5, i=33)),
    ("ab=iab,ib", dict(a=100, b=6, i=50)),
    ("a=iat,i", dict(a=300, i=20, t=7)),
    ("ab=ai,ibt", dict(a=130, b=70, i=9, t=3)),
    ("abc=aict,ibcs", dict(a=40, b=30, c=3, i=10, t=2, s=3)),
    ("bc=tbc,sbc", dict(b=20, c=10, t=5, s=7)),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", GENERAL_SHAPES)
def test_fused_batch_and_trace_indices(dtype, spec, ext):
    rng = np.random.default_rng(29)
    A, B, C0 = wl.tensors(spec, ext, rng, "normal", with_c=True)
    p = _plan(spec, ext, dtype)
    assert p.variants() == []
    got = run(p, A, B, dtype=dtype)
    check(spec, ext, A, B, got, dtype)
    got = run(p, A, B, C0, alpha=-0.75, beta=2.0, dtype=dtype)
    check(spec, ext, A, B, got, dtype, C0=C0, alpha=-0.75, beta=2.0)


def test_fused_batch_and_trace_integer_exact():
    for spec, ext in GENERAL_SHAPES:
        A, B, C = wl.tensors(spec, ext, np.random.default_rng(33), integer=True, with_c=True)
        for dtype in ("f64", "f32"):
            p = _plan(spec, ext, dtype)
            got = run(p, A, B, C, alpha=1.0, beta=-2.0, dtype=dtype)
            check(spec, ext, A, B, got, dtype, C0=C, alpha=1.0, beta=-2.0, exact=True)


def test_batch_api_with_batch_and_trace_members():
    """A graph batch mixing ordinary members with batch- and trace-index ones."""
    import torch
    specs = [GENERAL_SHAPES[0], GENERAL_SHAPES[2], GENERAL_SHAPES[4], ("abc=ai,ibc", dict(a=50, b=30, c=7, i=40))]
    plans, host, dev = [], [], []
    for t, (spec, ext) in enumerate(specs):
        A, B, _ = wl.tensors(spec, ext, np.random.default_rng(40 + t), "normal")
        p = _plan(spec, ext)
        plans.append(p)
        host.append((spec, ext, A, B))
        dev.append((tc.to_device_fortran(A, torch.float64), tc.to_device_fortran(B, torch.float64),
                    tc.empty_fortran(p.shape("C"), torch.float64).fill_(float("nan"))))
    batch = tc.Batch(plans)
    As, Bs, Cs = zip(*dev)
    batch.contract(As, Bs, Cs)
    torch.cuda.synchronize()
    for (spec, ext, A, B), C in zip(host, Cs):
        check(spec, ext, A, B, C.cpu().numpy())


# Outer products (no summed index): one K position.  C's unit index from A
# runs the streaming kernel, a permuted C the matrix-core kernel.
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext,strides", [
    ("abc=ab,c", dict(a=300, b=5, c=7), None),
    ("bak=ab,k", dict(a=16, b=5, k=9), dict(C=[16 * 9, 9, 1])),
    ("ab=a,b", dict(a=70, b=130), dict(C=[130, 1])),
])
def test_fused_outer_product(dtype, spec, ext, strides):
    import torch
    A, B, C0 = wl.tensors(spec, ext, np.random.default_rng(41), "normal", with_c=True)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p = _plan(spec, ext, dtype, strides=strides)
    sC = p.strides["C"]
    shapeC = p.shape("C")
    span = 1 + sum((e - 1) * st for e, st in zip(shapeC, sC))
    dC = torch.as_strided(torch.zeros(span, dtype=tdt, device="cuda"), tuple(shapeC), tuple(sC))
    dC.copy_(torch.from_numpy(np.array(C0)))
    p.contract(tc.to_device_fortran(A, tdt), tc.to_device_fortran(B, tdt), dC, -0.5, 1.5)
    torch.cuda.synchronize()
    check(spec, ext, A, B, dC.double().cpu().numpy(), dtype, C0=C0, alpha=-0.5, beta=1.5)


def test_fused_mfma_integer_exact():
    spec, ext = "abc=ija,jbic", dict(a=70, b=20, c=9, i=13, j=17)
    A, B, C = wl.tensors(spec, ext, np.random.default_rng(5), integer=True, with_c=True)
    for dtype in ("f64", "f32"):
        p = _plan(spec, ext, dtype)
        got = run(p, A, B, C, alpha=1.0, beta=2.0, dtype=dtype)
        check(spec, ext, A, B, got, dtype, C0=C, alpha=1.0, beta=2.0, exact=True)


def test_explicit_strides():
    """Padded, permuted layouts given by strides (same memory, other order)."""
    torch = pytest.importorskip("torch")
    spec, ext = "abc=ija,jbic", dict(a=24, b=10, c=6, i=7, j=5)
    A, B, _ = wl.tensors(spec, ext, np.random.default_rng(8), "normal")
    ref = oracle.contract(spec, ext, A, B)
    # A stored as [a][j][i] with padding: strides i=1, j=8, a=8*6
    sA = [1, 8, 48]
    bufA = torch.zeros(48 * 24 + 64, dtype=torch.float64, device="cuda")
    dA = torch.as_strided(bufA, (7, 5, 24), sA)
    dA.copy_(torch.from_numpy(A))
    dB = tc.to_device_fortran(B, torch.float64)
    # C in C-order (last index fastest)
    sC = [60, 6, 1]
    dC = torch.full((24 * 60,), float("nan"), dtype=torch.float64, device="cuda")
    dCv = torch.as_strided(dC, (24, 10, 6), sC)
    p = _plan(spec, ext, strides=dict(A=sA, C=sC))
    infos = p.variants()
    for v in [tc.TC_VARIANT_FUSED] + list(range(0, 176, 7)):
        p.set_variant(v)
        dCv.fill_(float("nan"))
        if v >= 0 and not infos[v]["runs_on_gpu"]:
            # a copy of C with a contracted loop at or outside it among the
            # free loops: the GPU schedule refuses it
            with pytest.raises(tc.TcError) as e:
                p.contract(dA, dB, dCv, 1.0, 0.0)
            assert e.value.name == "TC_E_UNSUPPORTED"
            continue
        p.contract(dA, dB, dCv, 1.0, 0.0)
        torch.cuda.synchronize()
        err = oracle.normwise_rel_err(dCv.cpu().numpy(), ref)
        assert err <= 1e-12, (v, err)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_every_variant_case_study(dtype):
    """All 36 members of C_abc = A_ai B_ibc (Section 3 case study, a=b=c=64,
    i=8) against the oracle; integer data bit-exact."""
    w = wl.smallk_cube(64, 8, integer=True)
    p = _plan(w["spec"], w["ext"], dtype)
    names = [v["name"] for v in p.variants()]
    assert len(names) == 36
    for v in range(36):
        p.set_variant(v)
        got = run(p, w["A"], w["B"], dtype=dtype)
        check(w["spec"], w["ext"], w["A"], w["B"], got, dtype, exact=True)


def test_every_variant_permuted_small():
    """All 176 members of C_abc = A_ija B_jbic (Section 4.3 Test 3) with ragged
    extents; integer data bit-exact, real data within tolerance, alpha/beta."""
    spec, ext = "abc=ija,jbic", dict(a=19, b=6, c=5, i=4, j=3)
    A, B, C = wl.tensors(spec, ext, np.random.default_rng(21), integer=True, with_c=True)
    p = _plan(spec, ext)
    assert len(p.variants()) == 176
    for v in range(176):
        p.set_variant(v)
        got = run(p, A, B, C, alpha=1.0, beta=-1.0)
        check(spec, ext, A, B, got, C0=C, alpha=1.0, beta=-1.0, exact=True)
    Ar, Br, _ = wl.tensors(spec, ext, np.random.default_rng(22), "normal")
    for v in range(0, 176, 5):
        p.set_variant(v)
        got = run(p, Ar, Br)
        check(spec, ext, Ar, Br, got)


def test_every_variant_other_patterns():
    for spec, ext in [("ab=iaj,jbi", dict(a=9, b=7, i=5, j=3)),
                      ("abcd=ai,ibcd", dict(a=6, b=3, c=4, d=2, i=5)),
                      ("a=iaj,ji", dict(a=11, i=6, j=4))]:
        A, B, _ = wl.tensors(spec, ext, np.random.default_rng(4), integer=True)
        p = _plan(spec, ext)
        for v in range(len(p.variants())):
            p.set_variant(v)
            got = run(p, A, B)
            check(spec, ext, A, B, got, exact=True)


def test_degenerate_extents():
    torch = pytest.importorskip("torch")
    # contracted extent 0: C = beta*C
    spec, ext = "abc=ai,ibc", dict(a=5, b=4, c=3, i=0)
    C0 = np.array(np.random.default_rng(1).uniform(-1, 1, (5, 4, 3)), order="F")
    p = _plan(spec, ext)
    got = run(p, np.zeros((5, 0), order="F"), np.zeros((0, 4, 3), order="F"), C0, alpha=1.0, beta=3.0)
    np.testing.assert_array_equal(got, 3.0 * C0)
    # empty output: no launch, no error
    p = _plan(spec, dict(a=0, b=4, c=3, i=2))
    dA = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    dB = tc.to_device_fortran(np.zeros((2, 4, 3)), torch.float64)
    dC = torch.zeros((0, 4, 3), dtype=torch.float64, device="cuda")
    p.contract(dA, dB, dC)
    # alpha = 0 reads neither input
    p = _plan(spec, dict(a=5, b=4, c=3, i=2))
    dC = tc.to_device_fortran(C0, torch.float64)
    tc.tc_contract(p.handle, 0, 0, dC.data_ptr(), 0.0, 2.0, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dC.cpu().numpy(), 2.0 * C0)


def test_alias_and_null_errors():
    torch = pytest.importorskip("torch")
    spec, ext = "ab=ai,ib", dict(a=8, b=8, i=8)
    p = _plan(spec, ext)
    buf = torch.zeros(64 * 3, dtype=torch.float64, device="cuda")
    with pytest.raises(tc.TcError) as e:
        tc.tc_contract(p.handle, buf.data_ptr(), buf.data_ptr() + 64 * 8, buf.data_ptr() + 32 * 8)
    assert e.value.name == "TC_E_ALIAS"
    with pytest.raises(tc.TcError) as e:
        tc.tc_contract(p.handle, 0, buf.data_ptr(), buf.data_ptr() + 128 * 8)
    assert e.value.name == "TC_E_NULL"


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("spec,ext", [
    ("bac=ai,ibc", dict(a=33, b=20, c=7, i=5)),
    ("bca=ija,jbic", dict(a=18, b=12, c=5, i=3, j=4)),
    ("bacd=ai,ibcd", dict(a=9, b=6, c=5, d=4, i=3)),
])
def test_members_copying_c(spec, ext, dtype):
    """Members that copy C's slice in before the call and out after it (Section
    2): per pass, a copy launch into a temporary, the body on the temporary, a
    copy launch back.  Every member of specs with such members, with alpha and
    beta, integer data, bit-exact against the oracle; the members whose C copy
    has a contracted loop at or outside it among the free loops are refused."""
    A, B, C0 = wl.tensors(spec, ext, np.random.default_rng(41), integer=True, with_c=True)
    p = _plan(spec, ext, dtype)
    infos = p.variants()
    copying = [v for v in range(len(infos)) if any(t == "C" for t, _ in infos[v]["copies"])]
    assert copying
    ran = 0
    for v in range(len(infos)):
        p.set_variant(v)
        if not infos[v]["runs_on_gpu"]:
            with pytest.raises(tc.TcError) as e:
                run(p, A, B, C0, alpha=2.0, beta=-1.0, dtype=dtype)
            assert e.value.name == "TC_E_UNSUPPORTED"
            continue
        got = run(p, A, B, C0, alpha=2.0, beta=-1.0, dtype=dtype)
        check(spec, ext, A, B, got, dtype, C0=C0, alpha=2.0, beta=-1.0, exact=True)
        ran += v in copying
    assert ran >= 3
