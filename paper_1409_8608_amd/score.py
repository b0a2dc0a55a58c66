"""Score the performance model: predict every member of a contraction's
family with tc_predict, time every member on the device, and compare.

    python -m paper_1409_8608_amd.score "abc=ai,ibc" a=64,b=64,c=64,i=8 [--dtype f64] [--json out.json]
    python -m paper_1409_8608_amd.score "abc=ai,ibc" a=256,b=256,c=256,i=8 --chain "b=ib,i" b=1048576,i=64

With --chain the contraction is the first of a two-contraction chain run again
and again (the second runs its fused kernel in between, on tensors of its own):
members are timed alone and right after the second contraction, and predicted
with the paper's root assumption and with the chain's root gaps
(tc_chain_root_gaps); each pairing is scored.

Reported per contraction (the paper's goal is to single out the fastest
members without running them, Sections 3 and 4):
  hit          the predicted-fastest member measures within 5% of the fastest
  strict_hit   it is exactly the fastest
  spearman     rank correlation of predicted and measured times (all members)
  median_rel   median |predicted - measured| / measured
  efficiency   sum of measured member times / time spent predicting
for each of the five prediction stages.  Each member is timed with HIP events,
median of up to five runs after one warm-up (one run if a member takes longer
than 0.2 s); inputs uniform[-1, 1] from a seeded generator.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def _spearman(x, y):
    rx = np.argsort(np.argsort(x)).astype(float)
    ry = np.argsort(np.argsort(y)).astype(float)
    if rx.std() == 0 or ry.std() == 0:
        return float("nan")
    return float(np.corrcoef(rx, ry)[0, 1])


def _time_members(p, ids, dA, dB, dC, cap_s, before=None):
    """Median of up to five timed runs per member; `before` runs ahead of each."""
    import torch

    import paper_1409_8608_amd as tc
    meas = []
    for v in ids:
        p.set_variant(v)
        try:
            p.contract(dA, dB, dC)
        except tc.TcError:
            meas.append(float("inf"))
            continue
        torch.cuda.synchronize()
        ts = []
        for _ in range(5):
            if before is not None:
                before()
            s, e = torch.cuda.Event(True), torch.cuda.Event(True)
            s.record()
            p.contract(dA, dB, dC)
            e.record()
            torch.cuda.synchronize()
            ts.append(s.elapsed_time(e) * 1e-3)
            if ts[-1] > cap_s:
                break
        meas.append(float(np.median(ts)))
    return np.array(meas)


def _pairing(names, preds, meas, stage=5):
    ok = np.isfinite(meas)
    best = float(meas[ok].min())
    pred = np.array([q["stage_s"][stage - 1] for q in preds])
    pk = int(np.argmin(np.where(ok, pred, np.inf)))
    rel = np.abs(pred[ok] - meas[ok]) / meas[ok]
    return dict(pick=names[pk], pick_over_best=float(meas[pk] / best), spearman=_spearman(pred[ok], meas[ok]),
                median_rel=float(np.median(rel)))


def score_chain(spec: str, extents: dict, qspec: str, qextents: dict, dtype: str = "f64", seed: int = 0,
                cap_s: float = 0.2):
    import torch

    import paper_1409_8608_amd as tc
    from paper_1409_8608_amd import workloads as wl
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p = tc.Plan(spec, extents, dtype)
    q = tc.Plan(qspec, qextents, dtype)
    preds0 = p.predict()
    tc.tc_chain_root_gaps([p.handle, q.handle], [1, 2, 3, 4, 5, 6])
    preds1 = p.predict()
    A, B, _ = wl.tensors(spec, extents, np.random.default_rng(seed), "uniform")
    dA, dB = tc.to_device_fortran(A, tdt), tc.to_device_fortran(B, tdt)
    dC = tc.empty_fortran(p.shape("C"), tdt)
    qA, qB, _ = wl.tensors(qspec, qextents, np.random.default_rng(seed + 1), "uniform")
    eA, eB = tc.to_device_fortran(qA, tdt), tc.to_device_fortran(qB, tdt)
    eC = tc.empty_fortran(q.shape("C"), tdt)
    names = [v["name"] for v in p.variants()] + ["fused"]
    ids = list(range(len(names) - 1)) + [tc.TC_VARIANT_FUSED]
    alone = _time_members(p, ids, dA, dB, dC, cap_s)
    chain = _time_members(p, ids, dA, dB, dC, cap_s, before=lambda: q.contract(eA, eB, eC))
    ok = np.isfinite(alone) & np.isfinite(chain)
    ratio_meas = chain[ok] / alone[ok]
    p0 = np.array([x["predicted_s"] for x in preds0])[ok]
    p1 = np.array([x["predicted_s"] for x in preds1])[ok]
    return dict(spec=spec, extents=extents, chain_with=qspec, chain_extents=qextents, dtype=dtype,
                members=len(names),
                measured_chain_over_alone=dict(median=float(np.median(ratio_meas)), min=float(ratio_meas.min()),
                                               max=float(ratio_meas.max())),
                predicted_gaps_over_default=dict(median=float(np.median(p1 / p0)), min=float((p1 / p0).min()),
                                                 max=float((p1 / p0).max())),
                alone_vs_default=_pairing(names, preds0, alone), chain_vs_default=_pairing(names, preds0, chain),
                chain_vs_gaps=_pairing(names, preds1, chain))


def score(spec: str, extents: dict, dtype: str = "f64", seed: int = 0, cap_s: float = 0.2):
    import torch

    import paper_1409_8608_amd as tc
    from paper_1409_8608_amd import workloads as wl
    tdt = torch.float64 if dtype == "f64" else torch.float32
    p = tc.Plan(spec, extents, dtype)
    t0 = time.perf_counter()
    preds = p.predict()
    t_predict = time.perf_counter() - t0
    A, B, _ = wl.tensors(spec, extents, np.random.default_rng(seed), "uniform")
    dA, dB = tc.to_device_fortran(A, tdt), tc.to_device_fortran(B, tdt)
    dC = tc.empty_fortran(p.shape("C"), tdt)
    names = [v["name"] for v in p.variants()] + ["fused"]
    ids = list(range(len(names) - 1)) + [tc.TC_VARIANT_FUSED]
    meas = _time_members(p, ids, dA, dB, dC, cap_s)
    ok = np.isfinite(meas)
    best = float(meas[ok].min())
    res = dict(spec=spec, extents=extents, dtype=dtype, members=len(names), predict_s=t_predict,
               fastest=names[int(np.argmin(np.where(ok, meas, np.inf)))], fastest_s=best, stages=[])
    for st in range(5):
        pred = np.array([q["stage_s"][st] for q in preds])
        pk = int(np.argmin(np.where(ok, pred, np.inf)))
        rel = np.abs(pred[ok] - meas[ok]) / meas[ok]
        res["stages"].append(dict(stage=st + 1, pick=names[pk], hit=bool(meas[pk] <= 1.05 * best),
                                  strict_hit=bool(meas[pk] == best), spearman=_spearman(pred[ok], meas[ok]),
                                  median_rel=float(np.median(rel))))
    res["efficiency"] = float(meas[ok].sum() / max(t_predict, 1e-9))
    res["per_member"] = [dict(name=n, measured_s=float(m), predicted_s=float(q["predicted_s"]))
                         for n, m, q in zip(names, meas, preds)]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("spec")
    ap.add_argument("extents", help="comma list like a=64,b=64,c=64,i=8")
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--json", default=None)
    ap.add_argument("--chain", nargs=2, metavar=("SPEC", "EXTENTS"), default=None,
                    help="score as the first contraction of a chain with this second one")
    args = ap.parse_args()
    ext = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.extents.split(",")}
    if args.chain:
        qext = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.chain[1].split(",")}
        r = score_chain(args.spec, ext, args.chain[0], qext, args.dtype)
        print(json.dumps(r), flush=True)
        if args.json:
            with open(args.json, "w") as f:
                json.dump(r, f)
        return
    r = score(args.spec, ext, args.dtype)
    line = {k: v for k, v in r.items() if k != "per_member"}
    print(json.dumps(line), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(r, f)


if __name__ == "__main__":
    main()
