"""Benchmark: contraction GFLOP/s and roofline fraction on one MI355X.

Headline workload (the metric's sweep, largest point): C_abc = A_ai B_ibc,
a = b = c = 1024, i = 8, FP64, column-major, entries uniform[-1, 1] (seed 28),
computed by the fused kernel.  One step = one tc_contract (plan and workspace
are set up before the timed region; inputs are resident in HBM).  Before the
--warmup steps the contraction runs for a fixed settling period (about 100
launches): on a fresh MI355X the launch time of this kernel falls from 3.7 ms
to 1.34 ms over its first 30 or so launches whatever ran before, so a short
warm-up alone would time the device's ramp rather than the kernel.

Printed: ONE JSON line with the headline value plus
  roofline      the dominant kernel's achieved algorithmic bandwidth (bytes of
                A + B + C once each / average launch time from HIP events on
                the launch stream) against the 8 TB/s HBM peak
  cpu_baseline  the FP64 oracle (plain C loop nest) on a bounded slab of the
                same workload, on all host cores (the primary value) and on
                one; the error of the timed GPU result against the oracle on
                the slab both computed; host CPU model and thread count; the
                paper's own flops/cycle figures and the GPU's flops/cycle at
                its measured engine clock
  forms         the other forms of the metric on the same GPU, each with its
                own roofline and its own fixed warm-up: FP64/FP32 fused
                permuted contraction, FP64/FP32 and split-BF16/FP8 matrix
                products, batched launch, complex storage; their sampled error
                columns compare against an FP64 numpy.einsum of the sampled
                slices (the oracle runs in the CPU-baseline leg only; the GPU
                parity tests check these configurations against it)
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


SETTLE_MS = 150.0      # settling period before the warm-up steps


def settle(fn, torch, ms=SETTLE_MS):
    """Run ``fn`` until ``ms`` of device time have passed; returns the launches."""
    t0 = time.perf_counter()
    n = 0
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(10):
            fn()
        n += 10
        torch.cuda.synchronize()
    return n


def gpu_sclk_mhz(fn, torch):
    """Engine clock (MHz) reported by rocm-smi while ``fn`` runs back to back
    (outside the timed region); None if rocm-smi gives no reading."""
    import re
    import subprocess
    import threading
    stop = threading.Event()

    def busy():
        while not stop.is_set():
            for _ in range(20):
                fn()
            torch.cuda.synchronize()
    th = threading.Thread(target=busy)
    th.start()
    try:
        time.sleep(0.2)
        out = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True, timeout=20).stdout
    except (OSError, subprocess.SubprocessError):
        out = ""
    finally:
        stop.set()
        th.join()
    vals = [int(v) for line in out.splitlines() if "sclk" in line.lower()
            for v in re.findall(r"(\d+)\s*Mhz", line, flags=re.I)]
    return max(vals) if vals else None


def headline(args, torch, tc, wl):
    n, i = args.n, 8
    w = wl.smallk_cube(n, i)
    spec, ext = w["spec"], w["ext"]
    plan = tc.Plan(spec, ext, "f64")
    plan.set_variant(tc.TC_VARIANT_FUSED)
    dA = tc.to_device_fortran(w["A"], torch.float64)
    dB = tc.to_device_fortran(w["B"], torch.float64)
    dC = tc.empty_fortran(plan.shape("C"), torch.float64)
    fn = lambda: plan.contract(dA, dB, dC, 1.0, 0.0)
    settled = settle(fn, torch)
    ms, wall = _events_time(fn, args.steps, args.warmup, torch)
    flops = 2 * n * n * n * i
    bytes_alg = 8 * (n * i + i * n * n + n * n * n)
    # the timed result's first slabs C[:, :, 0:8], for the CPU-baseline leg's
    # comparison with the oracle
    import numpy as np
    gpu_slab = dC[:, :, :HEADLINE_CHECK_SLABS].cpu().numpy()
    ok = bool(np.isfinite(gpu_slab).all())
    sclk = gpu_sclk_mhz(fn, torch)
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
        settle=dict(launches=settled, ms=SETTLE_MS, note="untimed launches before the warm-up steps"),
        finite=ok,
        gpu_clock=dict(sclk_mhz_measured=sclk, peak_mhz=2400,
                       flops_per_cycle_at_measured=round(flops / (ms * 1e-3) / (sclk * 1e6), 1) if sclk else None,
                       flops_per_cycle_at_peak_clock=round(flops / (ms * 1e-3) / 2.4e9, 1)),
    )
    del dC
    torch.cuda.empty_cache()
    return rec, w, gpu_slab


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


HEADLINE_CHECK_SLABS = 8

# The paper's own figures (FP64, x86, BLAS), context for the oracle's rate:
# flops per cycle as its text states them.
PAPER_FLOPS_PER_CYCLE = [
    dict(value=60, peak=80, what="best Test 3 gemm members (i'c-gemm, i'b-gemm), C_abc = A_ija B_jbic",
         hardware="10-core Ivy Bridge-EP E5-2680 v2, 10 threads, OpenBLAS", source="Section 4.3"),
    dict(value=20, peak=80, what="slowest Test 3 gemm member (jb'-gemm), same setting", source="Section 4.3"),
    dict(value=None, peak=8, what="per-core peak, Test 1 (C_abc = A_ai B_ibc, a=b=c=128, i swept)",
         hardware="Ivy Bridge-EP E5-2680 v2, one core, MKL", source="Section 4.1"),
    dict(value=None, peak=4, what="per-core peak, Section 3 case study (C_abc = A_ai B_ibc, i=8)",
         hardware="Harpertown E5450, one core, OpenBLAS", source="Section 3"),
]


def host_threads():
    """Host threads the CPU leg may use: this process's CPU affinity, capped by
    OMP_NUM_THREADS when set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, seconds, gpu_slab, gpu_rec):
    """The oracle as it stands on slabs C[:, :, 0:s] of the workload, on all
    host threads (C's outermost index spread over them) and on one: a short run
    gives the rate, then one run is sized to about `seconds`.  The all-thread
    run always covers C[:, :, 0:8], which the GPU's timed result is compared
    with."""
    import numpy as np
    import oracle
    n, i = w["ext"]["a"], w["ext"]["i"]

    def run(s, threads):
        B = np.asfortranarray(w["B"][:, :, :s])
        t0 = time.perf_counter()
        C = oracle.contract("abc=ai,ibc", dict(a=n, b=n, c=s, i=i), w["A"], B, threads=threads)
        return time.perf_counter() - t0, C

    def leg(threads, s_min, s_max):
        probe = min(n, max(2, threads))              # one slab per thread gives the rate
        dt0, _ = run(probe, threads)
        s = int(max(s_min, min(s_max, round(probe * seconds / max(dt0, 1e-6)))))
        dt, C = run(s, threads)
        fl = 2 * n * n * s * i
        return dict(value=round(fl / dt / 1e9, 4), seconds=round(dt, 2), slabs=s, gflop=round(fl / 1e9, 2)), C

    threads = host_threads()
    allc, C = leg(threads, HEADLINE_CHECK_SLABS, min(n, 256))
    err = _normwise(gpu_slab, C[:, :, :HEADLINE_CHECK_SLABS])
    del C
    one, _ = leg(1, 1, n)
    ghz = 2.4
    return dict(value=allc["value"], unit="GFLOP/s", cores=threads, kind="oracle",
                sample=f"C[:, :, 0:{allc['slabs']}] of the a=b=c={n}, i={i} workload ({allc['gflop']} GFLOP in "
                       f"{allc['seconds']} s, plain FP64 loop nest, C's outermost index over {threads} threads)",
                one_core=dict(value=one["value"], unit="GFLOP/s", cores=1,
                              sample=f"C[:, :, 0:{one['slabs']}] ({one['gflop']} GFLOP in {one['seconds']} s)"),
                host=dict(cpu_model=cpu_model(), cpu_count=os.cpu_count(), threads_used=threads),
                gpu_result_error=dict(normwise_vs_oracle=err, tolerance=1e-12,
                                      slab=f"C[:, :, 0:{HEADLINE_CHECK_SLABS}] of the timed result"),
                speedup_gpu_over_oracle=round(gpu_rec["value"] / allc["value"], 1),
                paper_flops_per_cycle=PAPER_FLOPS_PER_CYCLE,
                gpu_flops_per_cycle=gpu_rec["gpu_clock"])


FORMS = ("permuted", "precision", "batched", "complex")
# Each form settles for 100 ms, then takes its own warm-up and timed launches,
# independent of the headline's --steps / --warmup.
FORM_WARMUP, FORM_STEPS = 10, 20


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
        fn = lambda: plan.contract(dA, dB, dC)
        settle(fn, torch, 100.0)
        ms, _ = _events_time(fn, FORM_STEPS, FORM_WARMUP, torch)
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
    if "batched" in chosen:
        # the batched mixed-precision form: FP64 data, split-BF16 products
        out["batched_bf16x3"] = batched(args, torch, tc, wl, "f64", compute="bf16x3",
                                        sequential_ms=out["batched_f64"]["sequential_ms"])
        print("# batched bf16x3 done", file=sys.stderr, flush=True)
    if "complex" in chosen:
        out.update(complex_forms(args, torch, tc, wl))
        print("# complex done", file=sys.stderr, flush=True)
    if "batched_f32" in out and "batched_f64" in out:
        out["batched_f32"]["factor_vs_sequential_fp64"] = round(
            out["batched_f64"]["sequential_ms"] / out["batched_f32"]["batched_tuned_ms"], 3)
    if "batched_bf16x3" in out:
        out["batched_bf16x3"]["factor_vs_sequential_fp64"] = out["batched_bf16x3"]["speedup_vs_sequential"]
    return out


def batched(args, torch, tc, wl, dtype, compute="native", sequential_ms=None):
    """4096 contractions of the four batch patterns, uneven extents: one
    tc_contract per member on one stream versus one graph replay (before and
    after tuning).  Device data from a seeded torch generator (uniform[-1,1]).
    With compute="bf16x3" every member runs split-BF16 tiles in the graph and
    the sequential FP64 time of the native run is given."""
    import numpy as np
    shapes, redraws = wl.batch_shapes(4096)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    es = 8 if dtype == "f64" else 4
    gen = torch.Generator(device="cuda")
    gen.manual_seed(51)
    plans, As, Bs, Cs = [], [], [], []
    flops = bytes_ = 0
    for it in shapes:
        p = tc.Plan(it["spec"], it["ext"], dtype, compute=compute)
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
    if sequential_ms is None:
        seq_ms, seq_wall = _events_time(seq, 2, 1, torch)
    else:
        seq_ms, seq_wall = sequential_ms, None
    t0 = time.perf_counter()
    batch = tc.Batch(plans)
    create_s = time.perf_counter() - t0
    bound = batch.bind(As, Bs, Cs)        # operands checked once; each replay is one library call
    run = lambda: batch.run(bound)
    bat_ms, _ = _events_time(run, 5, 3, torch)
    t0 = time.perf_counter()
    batch.tune(2)
    tune_s = time.perf_counter() - t0
    tuned_ms, _ = _events_time(run, 5, 3, torch)
    t0 = time.perf_counter()
    score = batch.score(256, 51)          # every candidate of 256 seeded members timed alone
    score_s = time.perf_counter() - t0
    on_members = sum(1 for t in range(len(plans)) if batch.choice(t)["variant"] >= 0)
    batch.run(bound)                      # C again from the tuned graph (tuning and scoring overwrite it)
    info = batch.info()
    # sampled parity of the last replay
    rng = np.random.default_rng(3)
    worst = 0.0
    for t in rng.choice(len(plans), 6, replace=False):
        it = shapes[t]
        ref = _einsum_ref(it["spec"], As[t].double().cpu().numpy(), Bs[t].double().cpu().numpy())
        worst = max(worst, _normwise(Cs[t].double().cpu().numpy(), ref))
    peak = BF16_PEAK_TFS if compute == "bf16x3" else FP64_PEAK_TFS if dtype == "f64" else FP32_PEAK_TFS
    executed = flops * (6 if compute != "native" else 1)     # six products in the split form
    bound_ms = max(executed / (peak * 1e12), bytes_ / (HBM_PEAK_GBS * 1e9)) * 1e3
    rec = dict(workload="4096 contractions from {abc=ai,ibc; abc=ija,jbic; ab=iaj,jbi; abcd=ai,ibcd}, free extents "
                        "logU[8,256], contracted logU[4,64], largest operand <= 2^24 elements, uniform[-1,1]"
                        + ("" if compute == "native" else f", {compute} products on FP64 data"),
               redraws=redraws, gflop=round(flops / 1e9, 2), gbytes=round(bytes_ / 1e9, 2),
               sequential_ms=round(seq_ms, 3), create_s=round(create_s, 2),
               batched_ms=round(bat_ms, 3), batched_tuned_ms=round(tuned_ms, 3),
               speedup_vs_sequential=round(seq_ms / tuned_ms, 3),
               tiles=info["tiles"], groups=info["groups"], normwise_err_sampled_max=worst,
               tune_s=round(tune_s, 2),
               tuner=dict(top_k=2, candidates=("(fused view | gemm members with all loops free) x 3 tile shapes"
                                               if compute == "native" else "fused view x 3 tile shapes"),
                          members_on_family_variants=on_members, score_s=round(score_s, 2),
                          score={k: (round(v, 4) if isinstance(v, float) else v) for k, v in score.items()}),
               **({} if seq_wall is None else dict(sequential_wall_ms=round(seq_wall, 3))),
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
            fn = lambda: plan.contract(dA, dB, dC, 1 + 0j, 0j)
            settle(fn, torch, 100.0)
            ms, _ = _events_time(fn, FORM_STEPS, FORM_WARMUP, torch)
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
    absab = _einsum_ref(w["spec"], np.abs(w["A"][:, rows, :]), np.abs(w["B"][:, cols, :]))
    dA = tc.to_device_fortran(w["A"], torch.float64)
    dB = tc.to_device_fortran(w["B"], torch.float64)
    base_ms = None
    # FP64 plain, FP32 plain (FP32-rounded inputs, FP32 matrix cores), and the
    # split-BF16 (six term products; ablations with three and nine) and
    # split-FP8 forms on the FP64 inputs; normwise and componentwise
    # (max |C - ref| / (|A||B|)) errors against an FP64 einsum of the sampled
    # slices
    for name, dtype, compute, peak, nprod in (("fp64", "f64", "native", FP64_PEAK_TFS, 1),
                                              ("fp32", "f32", "native", FP32_PEAK_TFS, 1),
                                              ("bf16x3", "f64", "bf16x3", BF16_PEAK_TFS, 6),
                                              ("bf16x3_p3", "f64", "bf16x3", BF16_PEAK_TFS, 3),
                                              ("bf16x3_p9", "f64", "bf16x3", BF16_PEAK_TFS, 9),
                                              ("fp8x3", "f64", "fp8x3", FP8_PEAK_TFS, 6)):
        tdt = torch.float64 if dtype == "f64" else torch.float32
        xA, xB = (dA, dB) if dtype == "f64" else (dA.to(tdt), dB.to(tdt))
        plan = tc.Plan(w["spec"], w["ext"], dtype, compute=compute,
                       products=nprod if compute == "bf16x3" else None)
        plan.prepare()
        dC = tc.empty_fortran(plan.shape("C"), tdt)
        fn = lambda: plan.contract(xA, xB, dC)
        settle(fn, torch, 100.0)
        ms, _ = _events_time(fn, FORM_STEPS, FORM_WARMUP, torch)
        got = dC[torch.as_tensor(rows, device="cuda")][:, torch.as_tensor(cols, device="cuda")].double().cpu().numpy()
        err = _normwise(got, ref)
        cerr = float(np.max(np.abs(got - ref) / absab))
        tfs = fl / (ms * 1e-3) / 1e12
        executed = fl * nprod
        rec = dict(workload="C_ab = A_iaj B_jbi, a=b=4096, i=j=64, normal(0,1) x logU[1e-3,1e3] per slice",
                   ms=round(ms, 4), effective_gflops=round(tfs * 1e3, 1), normwise_err_sampled=err,
                   componentwise_err_sampled=cerr, term_products=nprod if compute != "native" else None,
                   roofline=dict(bound="mfma", achieved=round(executed / (ms * 1e-3) / 1e12, 2), peak=peak,
                                 unit="TFLOP/s", frac=round(executed / (ms * 1e-3) / 1e12 / peak, 4),
                                 counts="executed MFMA flops (one per term product for the split forms)"))
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
    rec, w, gpu_slab = headline(args, torch, tc, wl)
    print(f"# headline done: {rec['value']} GFLOP/s", file=sys.stderr, flush=True)
    if not args.no_forms:
        rec["forms"] = forms(args, torch, tc, wl)
        print("# forms done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, gpu_slab, rec)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
