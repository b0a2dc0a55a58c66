"""GPU parity of every member of the 4096-contraction batch (patterns
abc=ai,ibc, abc=ija,jbic, ab=iaj,jbi, abcd=ai,ibcd; free extents log-uniform
in [8, 256], contracted in [4, 64]) in one graph replay, FP64 and FP32, each
on a sampled sub-block of its outputs that the oracle computes.  Every member
also writes all of its C (C starts NaN-filled).  Tolerances: FP64 normwise
<= 1e-12, FP32 <= 1e-5 against the oracle on the values the device holds;
the split-BF16 form on FP64 data <= 1e-5 against the FP64 oracle and
componentwise within the FP32-accumulation bound of the oracle's exactly
accumulated split result."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
tc = pytest.importorskip("paper_1409_8608_amd")
from paper_1409_8608_amd import workloads as wl  # noqa: E402


def _sample_subproblem(spec, ext, A, B, C, rng, per_index=3):
    """Sampled sub-contraction of one member: up to ``per_index`` values of
    every free index (always including the last one), the contracted indices
    whole.  Returns (sub-extents, A_sub, B_sub, C_sub) as float64 host arrays."""
    import torch
    sa, sb = spec.split("=")[1].split(",")
    sc = spec.split("=")[0]
    picks = {}
    for ch in sc:
        n = ext[ch]
        k = min(n, per_index)
        chosen = rng.choice(n - 1, k - 1, replace=False) if k > 1 else np.array([], dtype=int)
        picks[ch] = np.sort(np.append(chosen, n - 1)).astype(np.int64)

    def take(x, letters):
        for ax, ch in enumerate(letters):
            if ch in picks:
                x = x.index_select(ax, torch.as_tensor(picks[ch], device=x.device))
        return x.double().cpu().numpy()
    sub = dict(ext, **{ch: len(v) for ch, v in picks.items()})
    return sub, take(A, sa), take(B, sb), take(C, sc)


@pytest.mark.parametrize("dtype,compute", [("f64", "native"), ("f32", "native"), ("f64", "bf16x3")])
def test_batch_every_member(dtype, compute):
    """The 4096-contraction batch (patterns abc=ai,ibc, abc=ija,jbic,
    ab=iaj,jbi, abcd=ai,ibcd; free extents log-uniform in [8, 256], contracted
    in [4, 64]; uniform[-1, 1] from a seeded device generator) in one graph
    replay, FP64 and FP32, and in the split-BF16 form on FP64 data (per-slice
    scales are per free index, so a sampled sub-block keeps its slices whole):
    every member on a sampled sub-block of its outputs."""
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    shapes, _ = wl.batch_shapes(4096)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(51)
    plans, As, Bs, Cs = [], [], [], []
    for it in shapes:
        p = tc.Plan(it["spec"], it["ext"], dtype, compute=compute)
        plans.append(p)
        As.append(tc.empty_fortran(p.shape("A"), tdt).uniform_(-1, 1, generator=gen))
        Bs.append(tc.empty_fortran(p.shape("B"), tdt).uniform_(-1, 1, generator=gen))
        Cs.append(tc.empty_fortran(p.shape("C"), tdt).fill_(float("nan")))
    batch = tc.Batch(plans)
    batch.contract(As, Bs, Cs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(4096)
    # the split-BF16 form works at FP32 level (against the FP64 oracle on the FP64 inputs)
    tol = 1e-12 if dtype == "f64" and compute == "native" else 1e-5
    worst = 0.0
    for t, it in enumerate(shapes):
        assert bool(torch.isfinite(Cs[t]).all()), (t, it)
        sub, Ah, Bh, got = _sample_subproblem(it["spec"], it["ext"], As[t], Bs[t], Cs[t], rng)
        ref = oracle.contract(it["spec"], sub, np.asfortranarray(Ah), np.asfortranarray(Bh))
        err = oracle.normwise_rel_err(got, ref)
        worst = max(worst, err)
        assert err <= tol, (t, it["spec"], it["ext"], err)
        if compute == "bf16x3":
            from gpu_util import split_bound
            from oracle import split as osplit
            sa, sb = it["spec"].split("=")[1].split(",")
            K = int(np.prod([it["ext"][ch] for ch in sa if ch not in it["spec"].split("=")[0]]))
            ref_split = osplit.contract_split(it["spec"], sub, np.asfortranarray(Ah), np.asfortranarray(Bh))
            absAB = oracle.contract(it["spec"], sub, np.abs(Ah), np.abs(Bh))
            assert np.all(np.abs(got - ref_split) <= split_bound(K) * absAB + 2.0 ** -52 * np.abs(ref_split)), t
    print(f"batch {dtype} {compute}: 4096 members, worst sampled normwise error {worst:.2e}")
    del batch, plans, As, Bs, Cs
    gc.collect()
    torch.cuda.empty_cache()
