"""Train the surrogate ensemble and run the surrogate-in-the-loop sweep.

    python -m paper_2207_06908_amd.surrogate_run train --out DIR [--cases 20000 --holdout 2000]
    python -m paper_2207_06908_amd.surrogate_run sweep --weights FILE [--queries 65536 --audit 512]

train: draws seeded electrode cases from the sweep ranges, computes their
GPR waveforms with the batched FDTD engine, trains four independently seeded
nets (BF16 MFMA kernels, Adam from lr 1e-3 with a cosine decay, batch 256,
150 epochs; --batch 1024 --epochs 50 gives the shorter schedule, which
stops short of 2% peak error on about one case in eight) and evaluates them
on held-out FDTD cases.  Writes DIR/surrogate_weights.npz and
DIR/train.json.

sweep: draws queries from ranges 20% wider than the training ranges (10% on
each side), answers them with one batched ensemble inference, sends the
queries whose nets disagree on the peak by more than the threshold to the
batched FDTD engine, and audits a random subset against FDTD.  Writes one JSON
line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def _log(msg):
    print(msg, flush=True)


def _summary(err):
    err = np.asarray(err)
    if err.size == 0:
        return {"n": 0}
    return {"n": int(err.size), "median": float(np.median(err)), "p95": float(np.percentile(err, 95)),
            "max": float(err.max()), "frac_le_2pct": float(np.mean(err <= 0.02))}


def train(a):
    import torch
    from . import scenarios as S
    from . import surrogate as U
    os.makedirs(a.out, exist_ok=True)
    cases = S.draw_cases(a.cases + a.holdout, a.seed)
    X = U.features(cases)
    scale = U.resistance_scale(cases)
    if a.dataset:   # waveforms of the same seeded cases from an earlier run
        d = np.load(a.dataset)
        assert np.array_equal(d["scale"], scale), "dataset was made from other cases"
        Y = d["Y"]
        gpr = Y.astype(np.float64) * scale[:, None]
        fd = json.load(open(os.path.join(os.path.dirname(a.dataset), "train.json")))["fdtd"]
        run = U.FdtdRun(None, fd["gpu_s"] * 1e3, fd["wall_s"], fd["cells"])
    else:
        _log(f"fdtd: {len(cases)} cases")
        run = U.run_fdtd(cases, chunk=a.chunk, log=_log)
        _log(f"fdtd done: {run.gpu_ms / 1e3:.1f} s GPU, {run.wall_s:.1f} s wall, "
             f"{len(cases) / (run.gpu_ms / 1e3):.1f} cases/s")
        gpr = U.resample(run.gpr)
        Y = (gpr / scale[:, None]).astype(np.float32)
        np.savez_compressed(os.path.join(a.out, "dataset.npz"), X=X, Y=Y, scale=scale)
    tr, te = slice(0, a.cases), slice(a.cases, a.cases + a.holdout)
    sur = U.Surrogate(n_nets=a.nets)
    sur.init([a.seed * 100 + 40 + q for q in range(a.nets)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = sur.train(X[tr], Y[tr], epochs=a.epochs, batch=a.batch, lr=a.lr, lr_min=a.lr_min, seed=a.seed,
                       log=_log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = a.nets * a.epochs * ((a.cases + a.batch - 1) // a.batch)
    flop = 6.0 * sum(k * n for k, n in zip(U.WIDTHS[:-1], U.WIDTHS[1:])) * a.cases * a.epochs * a.nets
    sur.save(os.path.join(a.out, "surrogate_weights.npz"))
    # held-out evaluation: every net and the ensemble mean against FDTD
    ref = gpr[te]
    ev = {}
    preds = []
    for q in range(a.nets):
        p = U.gpr_from_prediction(sur.predict(X[te], q), cases[te])
        preds.append(p)
        ev[f"net{q}"] = {"peak": _summary(U.peak_error(p, ref)), "l2": _summary(U.l2_error(p, ref))}
    ym, sp, fb = sur.route(X[te], a.threshold)
    pm = U.gpr_from_prediction(ym, cases[te])
    acc = np.setdiff1d(np.arange(ref.shape[0]), fb)
    ev["ensemble_mean"] = {"peak": _summary(U.peak_error(pm, ref)), "l2": _summary(U.l2_error(pm, ref))}
    ev["ensemble_accepted"] = {"threshold": a.threshold, "fallback_fraction": float(fb.size / ref.shape[0]),
                               "peak": _summary(U.peak_error(pm[acc], ref[acc])),
                               "l2": _summary(U.l2_error(pm[acc], ref[acc]))}
    out = {"cases": a.cases, "holdout": a.holdout, "seed": a.seed, "nets": a.nets, "epochs": a.epochs,
           "batch": a.batch, "lr": a.lr, "lr_min": a.lr_min, "widths": U.WIDTHS,
           "fdtd": {"gpu_s": run.gpu_ms / 1e3, "wall_s": run.wall_s, "cells": run.cells,
                    "cases_per_s_gpu": len(cases) / (run.gpu_ms / 1e3)},
           "training": {"wall_s": t_train, "adam_steps": steps, "final_loss": losses[:, -1].tolist(),
                        "first_loss": losses[:, 0].tolist(),
                        "tflops_achieved": flop / t_train / 1e12},
           "holdout_eval": ev}
    with open(os.path.join(a.out, "train.json"), "w") as f:
        json.dump(out, f, indent=1)
    _log(json.dumps(out["holdout_eval"]["ensemble_accepted"]))
    _log(json.dumps(out["training"]))


def sweep(a):
    import torch
    from . import scenarios as S
    from . import surrogate as U
    cases = S.draw_cases(a.queries, a.seed, widen=0.1)
    X = U.features(cases)
    sur = U.Surrogate(n_nets=a.nets, max_rows=a.queries)  # one inference chunk
    sur.load(a.weights)
    xd = torch.from_numpy(X).cuda()
    sur.route(xd[:1024], a.threshold)                       # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    ens = sur.ens
    ym, sp, ids, cnt = ens.infer_route(xd, a.threshold)
    e1.record()
    torch.cuda.synchronize()
    infer_ms = e0.elapsed_time(e1)
    fb = ids[:int(cnt.item())].cpu().numpy()
    ym = ym.cpu().numpy()
    t_infer_wall = time.perf_counter() - t0
    _log(f"inference: {a.queries} queries x {a.nets} nets in {infer_ms:.2f} ms; {fb.size} fallbacks")
    fb_cases = [cases[i] for i in fb]
    run_fb = U.run_fdtd(fb_cases, chunk=a.chunk, log=_log) if fb_cases else None
    fb_ms = run_fb.gpu_ms if run_fb else 0.0
    answer = U.gpr_from_prediction(ym, cases)
    if run_fb:
        answer[fb] = U.resample(run_fb.gpr)
    # audit: random queries against FDTD
    rng = np.random.default_rng(a.seed + 1)
    aud = np.sort(rng.choice(a.queries, size=min(a.audit, a.queries), replace=False))
    run_a = U.run_fdtd([cases[i] for i in aud], chunk=a.chunk, log=_log)
    ref = U.resample(run_a.gpr)
    is_fb = np.isin(aud, fb)
    pe = U.peak_error(answer[aud], ref)
    fdtd_cps = aud.size / (run_a.gpu_ms / 1e3)
    loop_cps = a.queries / ((infer_ms + fb_ms) / 1e3)
    out = {"queries": a.queries, "nets": a.nets, "threshold": a.threshold,
           "fallback_fraction": fb.size / a.queries,
           "inference_ms": infer_ms, "inference_cases_per_s": a.queries / (infer_ms / 1e3),
           "fallback_fdtd_ms": fb_ms, "surrogate_in_loop_cases_per_s": loop_cps,
           "fdtd_cases_per_s": fdtd_cps, "gain_vs_fdtd": loop_cps / fdtd_cps,
           "audit": {"n": int(aud.size), "fallbacks": int(is_fb.sum()),
                     "accepted_peak": _summary(pe[~is_fb]),
                     "accepted_l2": _summary(U.l2_error(answer[aud][~is_fb], ref[~is_fb])),
                     "all_peak": _summary(pe),
                     "surrogate_only_peak": _summary(U.peak_error(U.gpr_from_prediction(ym[aud], [cases[i] for i in aud]), ref))},
           "wall_s": {"inference": t_infer_wall, "fallback_fdtd": run_fb.wall_s if run_fb else 0.0,
                      "audit_fdtd": run_a.wall_s}}
    print(json.dumps(out), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(out, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", required=True)
    t.add_argument("--cases", type=int, default=20000)
    t.add_argument("--holdout", type=int, default=2000)
    t.add_argument("--seed", type=int, default=4)
    t.add_argument("--nets", type=int, default=4)
    t.add_argument("--epochs", type=int, default=150)
    t.add_argument("--batch", type=int, default=256)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--lr-min", type=float, default=1e-5)
    t.add_argument("--dataset", default="", help="reuse the FDTD waveforms of an earlier run (same seed/sizes)")
    t.add_argument("--chunk", type=int, default=2048)
    t.add_argument("--threshold", type=float, default=0.02)
    s = sub.add_parser("sweep")
    s.add_argument("--weights", required=True)
    s.add_argument("--queries", type=int, default=65536)
    s.add_argument("--audit", type=int, default=512)
    s.add_argument("--seed", type=int, default=5)
    s.add_argument("--nets", type=int, default=4)
    s.add_argument("--threshold", type=float, default=0.02)
    s.add_argument("--chunk", type=int, default=2048)
    s.add_argument("--json", default="")
    a = ap.parse_args(argv)
    {"train": train, "sweep": sweep}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
