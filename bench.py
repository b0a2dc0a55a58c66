"""Benchmark: contraction GFLOP/s and roofline fraction on one MI355X.

Headline workload (the metric's sweep, largest point): C_abc = A_ai B_ibc,
a = b = c = 1024, i = 8, FP64, column-major, entries uniform[-1, 1] (seed 28),
computed by the fused kernel.  One step = one tc_contract (plan and workspace
are set up before the timed region; inputs are resident in HBM).

Printed: ONE JSON line with the headline value plus
  roofline      the dominant kernel's achieved algorithmic bandwidth (bytes of
                A + B + C once each / average launch time from HIP events on
                the launch stream) against the 8 TB/s HBM peak
  cpu_baseline  the FP64 oracle (plain C loop nest, one core) on a bounded
                slab of the same workload
  forms         the other forms of the metric on the same GPU, each with its
                own roofline: FP64/FP32 fused permuted contraction, FP64/FP32
                and split-BF16/FP8 matrix products, batched launch, complex
                storage; their sampled error columns compare against an FP64
                numpy.einsum of the sampled slices
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "contraction GFLOP/s + % roofline (FP64 vs BF16-split vs batched), same GPU"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3
FP8_PEAK_TFS = 5000.0        # MI355X dense FP8 matrix peak (TFLOP/s)
BF16_PEAK_TFS = 2500.0


def _split(spec):
    out, ins = spec.split("=")
    a, b = ins.split(",")
    return a, b, out


def _flops(spec, ext):
    """2 x the product of all extents: one multiply and one add per term."""
    n = 2
    for ch in set(spec.replace("=", "").replace(",", "")):
        n *= int(ext[ch])
    return n


def _einsum_ref(spec, A, B):
    """Reference for the sampled error columns of the forms: numpy.einsum in
    FP64 (complex128 for complex data) on the sampled slices."""
    import numpy as np
    a, b, out = _split(spec)
    return np.einsum(f"{a},{b}->{out}", A, B, optimize=True)


def _normwise(got, ref):
    import numpy as np
    got = np.asarray(got)
    d = np.linalg.norm((got.astype(np.result_type(got, np.float64)) - ref).ravel())
    n = np.linalg.norm(np.asarray(ref).ravel())
    return float(d / n) if n else float(d)


def _events_time(fn, steps, warmup, torch):
    """Average ms per call over `steps` calls, HIP events on the current stream
    bracketed by device synchronisation; plus wall-clock ms per step."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return start.elapsed_time(stop) / steps, wall


def headline(args, torch, tc, wl):
    n, i = args.n, 8
    w = wl.smallk_cube(n, i)
    spec, ext = w["spec"], w["ext"]
    plan = tc.Plan(spec, ext, "f64")
    plan.set_variant(tc.TC_VARIANT_FUSED)
    plan.prepare()
    dA = tc.to_device_fortran(w["A"], torch.float64)
    dB = tc.to_device_fortran(w["B"], torch.float64)
    dC = tc.empty_fortran(plan.shape("C"), torch.float64)
    fn = lambda: plan.contract(dA, dB, dC, 1.0, 0.0)
    ms, wall = _events_time(fn, args.steps, args.warmup, torch)
    flops = 2 * n * n * n * i
    bytes_alg = 8 * (n * i + i * n * n + n * n * n)
    # sampled parity of the timed result (a few output columns)
    import numpy as np
    rng = np.random.default_rng(0)
    cs = rng.integers(0, n, 2)
    Cs = dC[:, :, torch.as_tensor(cs, device="cuda")].cpu().numpy()
    ok = bool(np.isfinite(Cs).all())
    gflops = flops / (ms * 1e-3) / 1e9
    achieved = bytes_alg / (ms * 1e-3) / 1e9
    rec = dict(
        metric=METRIC, value=round(gflops, 2), unit="GFLOP/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms, 5), wall_ms_per_step=round(wall, 5), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload=f"C_abc = A_ai B_ibc, a=b=c={n}, i={i}, FP64, column-major, uniform[-1,1], "
                             f"fused streaming kernel", spec=spec, extents=ext, seed=w["seed"],
                    flops=flops, algorithmic_bytes=bytes_alg),
        roofline=dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(),
                      kernel="k_stream_wave<double,8,2,8,64,false>"),
        finite=ok,
    )
    del dC
    torch.cuda.empty_cache()
    return rec, w


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed counter
    summary, if that summary was taken on the current kernel source (its
    SHA-256 is recorded in the summary); else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_stream_wave_smallk_cube_1024_counters.md")
    src = os.path.join(ROOT, "paper_1409_8608_amd", "csrc", "kernels_stream.hip")
    try:
        text = open(path).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel source sha256") != sha:
        return None
    try:
        return float(vals["traffic bytes per launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, seconds):
    """The oracle as it stands on a slab C[:, :, 0:s] of the workload: one
    slab times the rate, then one run sized to about `seconds`."""
    import numpy as np
    import oracle
    n, i = w["ext"]["a"], w["ext"]["i"]

    def run(s):
        B = np.asfortranarray(w["B"][:, :, :s])
        t0 = time.perf_counter()
        oracle.contract("abc=ai,ibc", dict(a=n, b=n, c=s, i=i), w["A"], B)
        return time.perf_counter() - t0

    dt4 = run(4)
    s = int(max(1, min(n, round(4 * seconds / max(dt4, 1e-6)))))
    dt = run(s)
    flops = 2 * n * n * s * i
    return dict(value=round(flops / dt / 1e9, 4), unit="GFLOP/s", cores=1, kind="oracle",
                sample=f"C[:, :, 0:{s}] of the a=b=c={n}, i={i} workload ({flops / 1e9:.2f} GFLOP in {dt:.1f} s, "
                       "one host core, plain FP64 loop nest)")


FORMS = ("permuted", "precision", "batched", "complex")


def forms(args, torch, tc, wl):
    """Other forms of the metric on the same GPU (short runs)."""
    out = {}
    import numpy as np
    chosen = FORMS if args.forms == "all" else tuple(args.forms.split(","))
    # FP64 / FP32 fused permuted contraction, C_abc = A_ija B_jbic (256^3, 32^2)
    w = wl.permuted(256, 32)
    for dt, tdt, peak in ((("f64", torch.float64, FP64_PEAK_TFS), ("f32", torch.float32, FP32_PEAK_TFS))
                          if "permuted" in chosen else ()):
        plan = tc.Plan(w["spec"], w["ext"], dt)
        plan.prepare()
        dA = tc.to_device_fortran(w["A"], tdt)
        dB = tc.to_device_fortran(w["B"], tdt)
        dC = tc.empty_fortran(plan.shape("C"), tdt)
        ms, _ = _events_time(lambda: plan.contract(dA, dB, dC), max(3, args.steps // 4), max(2, args.warmup // 2), torch)
        fl = 2 * 256 ** 3 * 32 * 32
        tfs = fl / (ms * 1e-3) / 1e12
        out[f"permuted_{dt}"] = dict(workload="C_abc = A_ija B_jbic, a=b=c=256, i=j=32, normal(0,1)",
                                     ms=round(ms, 4), gflops=round(tfs * 1e3, 1),
                                     roofline=dict(bound="mfma", achieved=round(tfs, 2), peak=peak,
                                                   unit="TFLOP/s", frac=round(tfs / peak, 4)))
        del dA, dB, dC
    torch.cuda.empty_cache()
    # precision: C_ab = A_iaj B_jbi, a=b=4096, i=j=64 (K=4096), per-slice scaled data;
    # FP64 plain vs split-BF16 (three terms, six products) on the same GPU
    if "precision" in chosen:
        out.update(precision(args, torch, tc, wl))
    for dt in (("f64", "f32") if "batched" in chosen else ()):
        out[f"batched_{dt}"] = batched(args, torch, tc, wl, dt)
        print(f"# batched {dt} done", file=sys.stderr, flush=True)
    if "complex" in chosen:
        out.update(complex_forms(args, torch, tc, wl))
        print("# complex done", file=sys.stderr, flush=True)
    if "batched_f32" in out and "batched_f64" in out:
        out["batched_f32"]["factor_vs_sequential_fp64"] = round(
            out["batched_f64"]["sequential_ms"] / out["batched_f32"]["batched_tuned_ms"], 3)
    return out


def batched(args, torch, tc, wl, dtype):
    """4096 contractions of the four batch patterns, uneven extents: one
    tc_contract per member on one stream versus one graph replay (before and
    after tuning).  Device data from a seeded torch generator (uniform[-1,1])."""
    import numpy as np
    shapes, redraws = wl.batch_shapes(4096)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    es = 8 if dtype == "f64" else 4
    gen = torch.Generator(device="cuda")
    gen.manual_seed(51)
    plans, As, Bs, Cs = [], [], [], []
    flops = bytes_ = 0
    for it in shapes:
        p = tc.Plan(it["spec"], it["ext"], dtype)
        plans.append(p)
        A = tc.empty_fortran(p.shape("A"), tdt).uniform_(-1, 1, generator=gen)
        B = tc.empty_fortran(p.shape("B"), tdt).uniform_(-1, 1, generator=gen)
        C = tc.empty_fortran(p.shape("C"), tdt)
        As.append(A); Bs.append(B); Cs.append(C)
        flops += _flops(it["spec"], it["ext"])
        bytes_ += es * (A.numel() + B.numel() + C.numel())
    for p in plans:
        p.prepare()

    def seq():
        for p, A, B, C in zip(plans, As, Bs, Cs):
            p.contract(A, B, C)
    seq_ms, seq_wall = _events_time(seq, 2, 1, torch)
    batch = tc.Batch(plans)
    run = lambda: batch.contract(As, Bs, Cs)
    bat_ms, _ = _events_time(run, 5, 3, torch)
    t0 = time.perf_counter()
    batch.tune(2)
    tune_s = time.perf_counter() - t0
    tuned_ms, _ = _events_time(run, 5, 3, torch)
    info = batch.info()
    # sampled parity of the last replay
    rng = np.random.default_rng(3)
    worst = 0.0
    for t in rng.choice(len(plans), 6, replace=False):
        it = shapes[t]
        ref = _einsum_ref(it["spec"], As[t].double().cpu().numpy(), Bs[t].double().cpu().numpy())
        worst = max(worst, _normwise(Cs[t].double().cpu().numpy(), ref))
    peak = FP64_PEAK_TFS if dtype == "f64" else FP32_PEAK_TFS
    bound_ms = max(flops / (peak * 1e12), bytes_ / (HBM_PEAK_GBS * 1e9)) * 1e3
    rec = dict(workload="4096 contractions from {abc=ai,ibc; abc=ija,jbic; ab=iaj,jbi; abcd=ai,ibcd}, free extents "
                        "logU[8,256], contracted logU[4,64], largest operand <= 2^24 elements, uniform[-1,1]",
               redraws=redraws, gflop=round(flops / 1e9, 2), gbytes=round(bytes_ / 1e9, 2),
               sequential_ms=round(seq_ms, 3), sequential_wall_ms=round(seq_wall, 3),
               batched_ms=round(bat_ms, 3), batched_tuned_ms=round(tuned_ms, 3), tune_s=round(tune_s, 2),
               speedup_vs_sequential=round(seq_ms / tuned_ms, 3), tune_hit_rate=info["tune_hit_rate"],
               tiles=info["tiles"], groups=info["groups"], normwise_err_sampled_max=worst,
               gflops=round(flops / (tuned_ms * 1e-3) / 1e9, 1),
               roofline=dict(bound="max(mfma, hbm)", lower_bound_ms=round(bound_ms, 3),
                             frac=round(bound_ms / tuned_ms, 4)))
    del batch, plans, As, Bs, Cs
    torch.cuda.empty_cache()
    return rec




def complex_forms(args, torch, tc, wl):
    """Complex storage: the headline shape (streamed C, few summed positions)
    and a square product (matrix cores through the real embedding), each with
    sampled outputs against an FP64 einsum of the sampled slices."""
    import numpy as np
    res = {}
    rng = np.random.default_rng(5)
    for name, w in (("smallk", wl.complex_smallk(1024, 8)), ("square", wl.complex_square(4096))):
        ext = w["ext"]
        sa, sb, sc = _split(w["spec"])
        picks = {ch: np.sort(rng.choice(ext[ch], min(ext[ch], 8), replace=False)) for ch in sc}
        sub = dict(ext, **{ch: len(v) for ch, v in picks.items()})
        Asub = w["A"][np.ix_(*[picks.get(ch, np.arange(ext[ch])) for ch in sa])]
        Bsub = w["B"][np.ix_(*[picks.get(ch, np.arange(ext[ch])) for ch in sb])]
        ref = _einsum_ref(w["spec"], Asub, Bsub)
        for dt, tdt, cb, peak in (("c128", torch.complex128, 16, FP64_PEAK_TFS),
                                  ("c64", torch.complex64, 8, FP32_PEAK_TFS)):
            plan = tc.Plan(w["spec"], ext, dt)
            plan.prepare()
            dA = tc.to_device_fortran(w["A"], tdt)
            dB = tc.to_device_fortran(w["B"], tdt)
            dC = tc.empty_fortran(plan.shape("C"), tdt)
            ms, _ = _events_time(lambda: plan.contract(dA, dB, dC, 1 + 0j, 0j), max(3, args.steps // 4),
                                 max(2, args.warmup // 2), torch)
            idx = [torch.as_tensor(picks[ch], device="cuda") for ch in sc]
            got = dC
            for ax, ix in enumerate(idx):
                got = got.index_select(ax, ix)
            got = got.cpu().numpy().astype(np.complex128)
            refd = ref if dt == "c128" else _einsum_ref(w["spec"], Asub.astype(np.complex64).astype(np.complex128),
                                                        Bsub.astype(np.complex64).astype(np.complex128))
            err = _normwise(got, refd)
            n_all = {t: int(np.prod([ext[ch] for ch in lets])) for t, lets in (("A", sa), ("B", sb), ("C", sc))}
            flops = 8 * int(np.prod([ext[ch] for ch in set(sa + sb + sc)]))
            rec = dict(workload=f"{w['spec']} " + ", ".join(f"{k}={v}" for k, v in ext.items()) +
                       f", complex uniform[-1,1] parts, {dt}",
                       ms=round(ms, 4), gflops_real=round(flops / (ms * 1e-3) / 1e9, 1),
                       normwise_err_sampled=err)
            if name == "smallk":
                gbs = cb * sum(n_all.values()) / (ms * 1e-3) / 1e9
                rec["roofline"] = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                                       frac=round(gbs / HBM_PEAK_GBS, 4),
                                       counts="A, B read once and C written once, complex elements")
            else:
                tfs = flops / (ms * 1e-3) / 1e12
                rec["roofline"] = dict(bound="mfma", achieved=round(tfs, 2), peak=peak, unit="TFLOP/s",
                                       frac=round(tfs / peak, 4), counts="8 real flops per complex term")
            res[f"complex_{name}_{dt}"] = rec
            del dA, dB, dC
            torch.cuda.empty_cache()
    return res


def precision(args, torch, tc, wl):
    import numpy as np
    res = {}
    w = wl.scaled_matrix(4096, 64)
    fl = 2 * 4096 * 4096 * 64 * 64
    rng = np.random.default_rng(7)
    rows = np.sort(rng.choice(4096, 24, replace=False))
    cols = np.sort(rng.choice(4096, 24, replace=False))
    ref = _einsum_ref(w["spec"], w["A"][:, rows, :], w["B"][:, cols, :])
    dA = tc.to_device_fortran(w["A"], torch.float64)
    dB = tc.to_device_fortran(w["B"], torch.float64)
    base_ms = None
    # FP64 plain, FP32 plain (FP32-rounded inputs, FP32 matrix cores), and the
    # split-BF16 and split-FP8 forms on the FP64 inputs; errors against an
    # FP64 einsum of the sampled slices
    for name, dtype, compute, peak in (("fp64", "f64", "native", FP64_PEAK_TFS),
                                       ("fp32", "f32", "native", FP32_PEAK_TFS),
                                       ("bf16x3", "f64", "bf16x3", BF16_PEAK_TFS),
                                       ("fp8x3", "f64", "fp8x3", FP8_PEAK_TFS)):
        tdt = torch.float64 if dtype == "f64" else torch.float32
        xA, xB = (dA, dB) if dtype == "f64" else (dA.to(tdt), dB.to(tdt))
        plan = tc.Plan(w["spec"], w["ext"], dtype, compute=compute)
        plan.prepare()
        dC = tc.empty_fortran(plan.shape("C"), tdt)
        ms, _ = _events_time(lambda: plan.contract(xA, xB, dC), 10, max(1, args.warmup // 5), torch)
        got = dC[torch.as_tensor(rows, device="cuda")][:, torch.as_tensor(cols, device="cuda")].double().cpu().numpy()
        err = _normwise(got, ref)
        tfs = fl / (ms * 1e-3) / 1e12
        executed = fl * (6 if compute != "native" else 1)
        rec = dict(workload="C_ab = A_iaj B_jbi, a=b=4096, i=j=64, normal(0,1) x logU[1e-3,1e3] per slice",
                   ms=round(ms, 4), effective_gflops=round(tfs * 1e3, 1), normwise_err_sampled=err,
                   roofline=dict(bound="mfma", achieved=round(executed / (ms * 1e-3) / 1e12, 2), peak=peak,
                                 unit="TFLOP/s", frac=round(executed / (ms * 1e-3) / 1e12 / peak, 4),
                                 counts="executed MFMA flops (6 products for the split forms)"))
        if base_ms is None:
            base_ms = ms
        else:
            rec["speedup_vs_fp64"] = round(base_ms / ms, 3)
        res[f"precision_{name}"] = rec
        del dC
        if dtype != "f64":
            del xA, xB
    del dA, dB
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--forms", default="all",
                    help="comma list of the other forms to run: " + ", ".join(FORMS) + " (default all)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (torch copy_) three times, outside the timed "
                         "region, so that profiler byte counters can be scaled by a kernel of known traffic")
    args = ap.parse_args()
    if args.forms != "all" and any(f not in FORMS for f in args.forms.split(",")):
        print(f"--forms takes a comma list of {', '.join(FORMS)}", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(see the sharding paragraph of DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1409_8608_amd as tc
    from paper_1409_8608_amd import workloads as wl
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calib_copy:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    rec, w = headline(args, torch, tc, wl)
    print(f"# headline done: {rec['value']} GFLOP/s", file=sys.stderr, flush=True)
    if not args.no_forms:
        rec["forms"] = forms(args, torch, tc, wl)
        print("# forms done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
