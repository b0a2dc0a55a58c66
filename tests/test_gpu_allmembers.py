"""GPU parity of every family member at the workloads' full sizes, on
sampled outputs that the oracle computes:
  - Test 3 (Section 4.3), C_abc = A_ija B_jbic at 256^3 x 32^2: all 176
    members, FP64, two sampled c-slabs each;
  - the headline size, C_abc = A_ai B_ibc at n = 1024, i = 8: all 36 members
    (8.6 GB outputs), two sampled c-slabs each;
  - Test 1 (Section 4.1), a = b = c = 128 with i = 16, 64, 256, 1024: all 36
    members at each i, two sampled c-slabs each.
Every member also writes all of C (C starts NaN-filled and must end finite).
Tolerance: FP64 normwise <= 1e-12 against the oracle."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
tc = pytest.importorskip("paper_1409_8608_amd")
from paper_1409_8608_amd import workloads as wl  # noqa: E402


def _dev(x):
    import torch
    return tc.to_device_fortran(x, torch.float64)


class _Members:
    """One contraction's device operands and oracle slabs C[..., c] for a few
    sampled values of C's last index.  Members run on a plan of their own per
    test (``plan()``): a member's copy temporaries stay with its plan, and
    some Test 3 members copy a slice once per parallel invocation (tens of GB
    at full size), so a plan shared by the whole module would hold the largest
    of them to the end."""

    def __init__(self, w, n_slabs, seed):
        import torch
        self.w = w
        self.dA, self.dB = _dev(w["A"]), _dev(w["B"])
        self.dC = tc.empty_fortran([w["ext"][ch] for ch in w["spec"].split("=")[0]], torch.float64)
        n_c = w["ext"]["c"]
        cs = np.random.default_rng(seed).choice(n_c - 1, n_slabs - 1, replace=False)
        self.cs = np.sort(np.append(cs, n_c - 1))             # always the last slab (ragged loop ends)
        sa, sb, _ = w["spec"].split("=")[1].split(",") + [None]
        Bs = np.asfortranarray(np.take(w["B"], self.cs, axis=sb.index("c")))
        self.ref = oracle.contract(w["spec"], dict(w["ext"], c=len(self.cs)), w["A"], Bs)

    def plan(self):
        return tc.Plan(self.w["spec"], self.w["ext"], "f64")

    def check(self, plan, v):
        import torch
        plan.set_variant(v)
        self.dC.fill_(float("nan"))
        plan.contract(self.dA, self.dB, self.dC)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(self.dC).all()), f"member {v}: part of C not written"
        pick = [v % len(self.cs), (v + 3) % len(self.cs)]
        got = self.dC[:, :, torch.as_tensor(self.cs[pick], device="cuda")].cpu().numpy()
        err = oracle.normwise_rel_err(got, self.ref[:, :, pick])
        assert err <= 1e-12, f"member {v} ({plan.variants()[v]['name']}): normwise error {err:.2e}"


@pytest.fixture(scope="module")
def test3_full():
    return _Members(wl.permuted(256, 32), 8, 31)


@pytest.mark.parametrize("chunk", range(11))
def test_test3_every_member_full_size(test3_full, chunk):
    """Test 3's 176 members at 256^3 x 32^2, sixteen per test."""
    plan = test3_full.plan()
    assert len(plan.variants()) == 176
    for v in range(16 * chunk, 16 * chunk + 16):
        test3_full.check(plan, v)


@pytest.fixture(scope="module")
def headline_full():
    return _Members(wl.smallk_cube(1024, 8), 6, 1024)


@pytest.mark.parametrize("chunk", range(4))
def test_headline_size_every_member(headline_full, chunk):
    """The 36 members of C_abc = A_ai B_ibc at n = 1024, i = 8, nine per test."""
    plan = headline_full.plan()
    assert len(plan.variants()) == 36
    for v in range(9 * chunk, 9 * chunk + 9):
        headline_full.check(plan, v)


@pytest.mark.parametrize("i", [16, 64, 256, 1024])
def test_test1_sweep_every_member(i):
    """Test 1's sweep over the contracted length: all 36 members at
    a = b = c = 128 for each i."""
    m = _Members(wl.smallk_cube(128, i), 4, i)
    plan = m.plan()
    for v in range(36):
        m.check(plan, v)
