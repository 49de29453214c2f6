"""Benchmark of the MI355X FDTD hot path.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--variant tuned|auto|split|fused|tb2]

Workload: the 512 x 512 x 384 Yee grid (dx 0.5 m, 10-cell CPML on all faces,
two-layer soil, 30 m thin wire driven by a 10 kA 1/50 us current, voltage
and field probes), synthetic and seeded.  A step is one full time step of
the hot path: H and E updates with lossy coefficients, CPML, thin-wire
classes, source injection and probe recording.  Inputs are resident in HBM
before timing starts.  Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# HBM bytes per launch of the dominant kernel from the profiler's FETCH_SIZE and
# WRITE_SIZE counters, scaled by what they read for a plain 1 GiB copy (x2.0
# and x1.0), keyed by the hash of the kernel sources they were taken with:
# once the kernels change the figure no longer applies and is reported null.
# the kernels, and the host code that builds their tile lists and launches
KERNEL_SOURCES = ("paper_2207_06908_amd/csrc/fdtd_kernels.hip", "paper_2207_06908_amd/csrc/fdtd_tile.h",
                  "paper_2207_06908_amd/csrc/fdtd_debye.hip", "paper_2207_06908_amd/csrc/yee_update.h",
                  "paper_2207_06908_amd/csrc/fdtd_dev.h", "paper_2207_06908_amd/csrc/fdtd_host.cpp")
MEASURED_TRAFFIC = {
    # (source hash, kernel variant, tile_y, tile_z): HBM bytes per step (all
    # launches of the step; a two-step pass counts half)
    ("bcecac58d1d08ec9", "tb2", 8, 20): 4.452e9,
    ("bcecac58d1d08ec9", "tb2", 8, 16): 4.471e9,
}


def kernel_source_hash() -> str:
    """sha256 (first 16 hex digits) of the kernel and launch sources with
    comments and white space removed, so that edits to comments keep the
    figures."""
    import hashlib
    import re
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # block comments
        text = re.sub(r"//[^\n]*", " ", text)                # line comments
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(steps: int):
    """Time the FP64 oracle on a bounded sample of the same workload: the
    full grid for a few steps (set-up excluded), on all the threads it is
    given and on one thread (a sixteenth of the steps)."""
    from oracle import orc
    from paper_2207_06908_amd import scenarios as S
    orc.build(force=False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    steps1 = max(3, steps // 16)
    sc = S.config2(n_steps=steps + steps1 + 1)
    o = orc.Oracle.from_params(sc.params())
    S.apply(sc, o)
    orc.set_threads(threads)
    o.step(1)  # builds the tables; not timed
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    orc.set_threads(1)
    t0 = time.perf_counter()
    o.step(steps1)
    dt1 = time.perf_counter() - t0
    orc.set_threads(threads)
    return {"value": sc.cells * steps / dt / 1e6, "unit": "Mcell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"FP64 oracle, full 512x512x384 grid, {steps} steps after table build",
            "cpu": _cpu_model(), "value_1_thread": sc.cells * steps1 / dt1 / 1e6,
            "sample_1_thread": f"the next {steps1} steps on one thread"}


def stream_ceiling(mib: int = 2048, reps: int = 10):
    """Practical HBM ceiling on this GPU: best of `reps` device copies
    (read + write) and triads a = b + s c (two reads, one write) of `mib` MiB
    arrays, timed with events."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.ones(n, dtype=torch.float32, device="cuda")
    c = torch.ones(n, dtype=torch.float32, device="cuda")
    def best(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1))
        return nbytes / (min(t) / 1e3) / 1e9
    copy = best(lambda: a.copy_(b), 8 * n)
    triad = best(lambda: torch.add(b, c, alpha=0.5, out=a), 12 * n)
    del a, b, c
    torch.cuda.empty_cache()
    return round(copy, 1), round(triad, 1)


def bench_batch(warmup: int = 100, graph_steps: int = 100, tune: bool = True):
    """The 256-grid electrode sweep (uneven 32-96^3 grids, dx 0.25 m, 8-cell
    CPML, 2000 steps) in the batched engine with HIP-graph replay; tile shape
    from the autotuner (cached) unless tune is False."""
    import torch
    from paper_2207_06908_amd import autotune
    from paper_2207_06908_amd import fdtd
    from paper_2207_06908_amd import scenarios as S
    steps = 2000
    tune_steps = autotune.tuning_steps(batch=True) if tune else 0
    scs = S.config3(n_steps=tune_steps + warmup + steps)
    grids = []
    for sc in scs:
        g = fdtd.Grid.from_params(sc.params(), precision=32)
        S.apply(sc, g)
        grids.append(g)
    tile = (32, 8, 32)
    persistent = True
    b = fdtd.Batch(grids, tile=tile, graph_steps=graph_steps)
    if tune:
        b.bind()
        c = autotune.tune_batch(b, autotune.batch_key([(s.nx, s.ny, s.nz) for s in scs], scs[0].npml))
        tile = (c["tile_x"], c["tile_y"], c["tile_z"])
        autotune.apply_batch(b, c, graph_steps)
        persistent = c.get("persistent", True)
    b.run(warmup)
    torch.cuda.synchronize()
    b.timing(True)
    b.run(steps)
    ms, n = b.time()
    cells = b.cells
    bytes_step = b.algorithmic_bytes_per_step()
    achieved = bytes_step * steps / (ms / 1e3) / 1e9
    out = {"workload": f"{len(scs)} independent electrode grids, 32-96^3 (x grown to fit the electrode), "
                       f"dx 0.25 m, 8-cell CPML, {steps} steps, HIP graph of {graph_steps} steps",
           "kernel": (("k_tb2_batch_q: two persistent work-queue launches per two-step pass (tiles clear of "
                        "the y slabs; the rest)" if persistent
                       else "k_tb2_batch: one launch per CPML group and two-step pass") if tile[0] == 60
                      else "k_fused_batch: one launch per step"),
           "tile": list(tile),
           "cells": cells, "value": round(cells * steps / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s",
           "cases_per_s": round(len(scs) / (ms / 1e3), 2), "ms_per_step": round(ms / steps, 5),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_step": bytes_step}}
    del b, grids
    torch.cuda.empty_cache()
    return out


def bench_debye(steps: int = 400, warmup: int = 20):
    """The 512 x 512 x 384 scene with the paper's measured four-pole Debye
    soil in both layers.  The autotuner picks, for this grid, between the
    split pass with polarisation currents and the fused pass over CPML tile
    groups (and its chunk height); the picked pass gives the value and the
    roofline, and both passes are timed and reported beside it."""
    import torch
    from paper_2207_06908_amd import autotune, fdtd
    from paper_2207_06908_amd import scenarios as S
    tune_steps = len(autotune.DEBYE_CANDIDATES) * (4 + 24)
    sc = S.config2_debye(n_steps=tune_steps + 2 * (warmup + steps) + 8)
    g = fdtd.Grid.from_params(sc.params(), precision=32)
    S.apply(sc, g)
    g.bind()
    choice = autotune.tune_grid(g, autotune.grid_key(sc.params()) + "/debye4", candidates=autotune.DEBYE_CANDIDATES)
    fused_tz = choice["tile_z"] if choice["variant"] == fdtd.KERNEL_FUSED else 32

    def timed(variant, ty, tz):
        g.set_kernel(variant, ty, tz)
        g.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g.timing(True)
        g.kernel_time()          # drains and resets
        e0.record()
        g.step(steps)
        e1.record()
        torch.cuda.synchronize()
        kms, kn = g.kernel_time()
        g.timing(False)
        return e0.elapsed_time(e1) / steps, kms / max(kn, 1)

    runs = {"split": timed(fdtd.KERNEL_SPLIT, 0, 0), "fused": timed(fdtd.KERNEL_FUSED, 8, fused_tz)}
    picked = "fused" if choice["variant"] == fdtd.KERNEL_FUSED else "split"
    ms, kms = runs[picked]
    bytes_step = g.algorithmic_bytes_per_step()
    achieved = bytes_step / (kms / 1e3) / 1e9
    kernels = {"split": "k_h_split + k_e_split_debye (two launches per step)",
               "fused": f"k_fused_list_debye (one launch per step and CPML tile group, {fused_tz}-plane chunks)"}
    out = {"workload": "512x512x384 Yee FDTD as above, both soil layers four-pole Debye soil "
                       "(eps_inf 16.381, sigma0 2.684 mS/m), ADE currents",
           "kernel": kernels[picked] + " (the autotuner's pick)",
           "cells": sc.cells, "steps": steps,
           "value": round(sc.cells / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s",
           "ms_per_step": round(ms, 5),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_step": bytes_step,
                        "kernel_ms_per_step": round(kms, 5)}}
    for name, (m, _k) in runs.items():
        out[name] = {"kernel": kernels[name], "ms_per_step": round(m, 5),
                     "value": round(sc.cells / (m / 1e3) / 1e6, 1)}
    del g
    torch.cuda.empty_cache()
    return out


def bench_lumped(steps: int = 1000, warmup: int = 20):
    """The 512 x 512 x 384 scene with a resistive voltage source and a lumped
    R and C: the same two-step pass (the elements are coefficient classes)."""
    import torch
    from paper_2207_06908_amd import fdtd
    from paper_2207_06908_amd import scenarios as S
    sc = S.config2_lumped(n_steps=warmup + steps)
    g = fdtd.Grid.from_params(sc.params(), precision=32)
    S.apply(sc, g)
    g.bind()
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out = {"workload": "512x512x384 Yee FDTD as above, source gap as a 400-ohm resistive voltage source, "
                       "1 kohm + 100 pF lumped at the wire base",
           "steps": steps, "value": round(sc.cells * steps / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s",
           "ms_per_step": round(ms / steps, 5), "coefficient_classes": g.num_classes}
    del g
    torch.cuda.empty_cache()
    return out


def bench_oblique(steps: int = 400, warmup: int = 20):
    """The 512 x 512 x 384 scene with a slanted 37-segment conductor: the
    two-step pass, with the wire's current, charge and source-amplitude
    kernels beside it."""
    import torch
    from paper_2207_06908_amd import fdtd
    from paper_2207_06908_amd import scenarios as S
    sc = S.config2_oblique(n_steps=warmup + steps)
    g = fdtd.Grid.from_params(sc.params(), precision=32)
    S.apply(sc, g)
    g.bind()
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out = {"workload": "512x512x384 Yee FDTD as above plus a slanted 5 cm conductor (20 x 12 x 30 cells, "
                       "37 segments), driven at its base",
           "kernel": "k_tb2_list (two-step pass over CPML groups; the wire's edges are sources whose amplitudes "
                     "k_owire_cur/k_owire_q/k_owire_amp/k_owire_e1 write on a third stream)",
           "steps": steps, "value": round(sc.cells * steps / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s",
           "ms_per_step": round(ms / steps, 5)}
    del g
    torch.cuda.empty_cache()
    return out


def bench_tower(steps: int = 400, warmup: int = 20):
    """The 512 x 512 x 384 scene with a lightning strike to a 30 m lattice
    tower of 15 oblique wires joined at 5 junctions (scenarios.config2_tower):
    the two-step pass with the wire kernels beside it."""
    import torch
    from paper_2207_06908_amd import fdtd
    from paper_2207_06908_amd import scenarios as S
    sc = S.config2_tower(n_steps=warmup + steps)
    g = fdtd.Grid.from_params(sc.params(), precision=32)
    S.apply(sc, g)
    g.bind()
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    segs = sum(g.oblique_wire_segments(w) for w in range(len(sc.owires)))
    out = {"workload": "512x512x384 Yee FDTD grid and soil as above; a 30 m lattice tower of oblique wires (4 legs "
                       f"cut at a ring, a 4-wire ring, 2 cross-arms; {len(sc.owires)} wires, {segs} segments, "
                       f"{len(sc.ojunctions)} junctions) struck through a channel wire by 10 kA 1/50 us",
           "kernel": "k_tb2_list (two-step pass over CPML groups; the wires' edges are sources written by "
                     "k_owire_cur/k_owire_q/k_owire_junc/k_owire_amp/k_owire_e1 on a third stream)",
           "steps": steps, "value": round(sc.cells * steps / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s",
           "ms_per_step": round(ms / steps, 5)}
    del g
    torch.cuda.empty_cache()
    return out


def bench_array(steps: int = 20000, warmup: int = 2000):
    """The apparent-resistivity array (100 x 100 x 80 cells, three Debye soil
    layers, Heidler source): a bounded window of its 4.2M-step run."""
    import torch
    from paper_2207_06908_amd import fdtd
    from paper_2207_06908_amd import scenarios as S
    sc = S.config_array(n_steps=warmup + steps)
    g = fdtd.Grid.from_params(sc.params(), precision=32)
    S.apply(sc, g)
    g.bind()
    g.set_graph(100)   # 800k cells: replay saves the host launch cost (a few percent here)
    g.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    full = sc.meta["full_steps"]
    out = {"workload": "apparent-resistivity array, 100x100x80 cells, dx 0.05 m, three 4-pole Debye layers, "
                       "8 thin wires, Heidler source; steps 2000-22000 of the 400 us run",
           "kernel": "k_h_split + k_e_split_debye + k_probes per step, replayed from 100-step HIP graphs",
           "steps": steps, "value": round(sc.cells * steps / (ms / 1e3) / 1e6, 1), "unit": "Mcell-updates/s",
           "ms_per_step": round(ms / steps, 6), "full_run_steps": full,
           "full_run_s": round(full * ms / steps / 1e3, 1)}
    del g
    torch.cuda.empty_cache()
    return out


def calibrate_copy(mib: int = 1024, reps: int = 3):
    """Plain device-to-device copies of known size, run under the profiler's
    FETCH_SIZE / WRITE_SIZE counters to scale them to true HBM bytes."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    for _ in range(reps):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy_ and neg", "bytes_read": 4 * n, "bytes_written": 4 * n,
                      "reps": reps}), flush=True)


def bench_surrogate(queries: int = 65536, audit: int = 512):
    """Surrogate in the loop on the electrode sweep: queries from ranges 20%
    wider than the training ranges, one batched inference of the 4-net
    ensemble with routing, fallback queries priced at the batched FDTD
    engine's measured cases/s on the audit cases.  Two routing rules:
    "fast" (spread of the nets' peaks > 2% -> FDTD) and "guarded" (also
    every query outside the training box, spread > 0.5%).  An audit of
    `audit` random queries runs through FDTD: the peak error of the answers
    delivered (the ensemble's where accepted, FDTD's where routed)."""
    import math
    import numpy as np
    import torch
    from paper_2207_06908_amd import scenarios as S
    from paper_2207_06908_amd import surrogate as U
    weights = os.path.join(ROOT, "paper_2207_06908_amd", "data", "surrogate_weights.npz")
    cases = S.draw_cases(queries, seed=5, widen=0.1)
    X = torch.from_numpy(U.features(cases)).cuda()
    aud = np.sort(np.random.default_rng(6).choice(queries, size=audit, replace=False))
    run = U.run_fdtd([cases[i] for i in aud])
    ref = U.resample(run.gpr)
    fdtd_cps = audit / (run.gpu_ms / 1e3)
    sur = U.Surrogate(n_nets=4, max_rows=queries)   # one chunk: the products take 128 x 128 tiles
    sur.load(weights)
    aud_t = torch.from_numpy(aud).cuda()
    points = {}
    for name, thr, bound in (("fast", U.FAST_THRESHOLD, math.inf), ("guarded", U.GUARD_THRESHOLD, U.GUARD_BOUND)):
        sur.guard(bound)
        sur.ens.infer_route(X, thr)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ym, _sp, ids, cnt = sur.ens.infer_route(X, thr)
        e1.record()
        torch.cuda.synchronize()
        infer_s = e0.elapsed_time(e1) / 1e3
        n_fb = int(cnt.item())
        fb = ids[:n_fb].cpu().numpy()
        answer = U.gpr_from_prediction(ym[aud_t].cpu().numpy(), [cases[i] for i in aud])
        is_fb = np.isin(aud, fb)
        answer[is_fb] = ref[is_fb]                  # routed queries are answered by the engine
        pe = U.peak_error(answer, ref)
        loop_s = infer_s + n_fb / fdtd_cps
        points[name] = {
            "spread_threshold": thr, "input_bound": None if math.isinf(bound) else bound,
            "inference_ms": round(infer_s * 1e3, 3), "fallback_fraction": round(n_fb / queries, 5),
            "surrogate_in_loop_cases_per_s": round(queries / loop_s, 1),
            "gain_vs_fdtd": round((queries / loop_s) / fdtd_cps, 1),
            "audit_delivered_peak_error": {"n": audit, "routed": int(is_fb.sum()),
                                           "median": round(float(np.median(pe)), 5),
                                           "p95": round(float(np.percentile(pe, 95)), 5),
                                           "max": round(float(pe.max()), 5),
                                           "frac_le_2pct": round(float(np.mean(pe <= 0.02)), 4)}}
        if name == "fast":
            fast_infer_s = infer_s
    w = U.WIDTHS
    flop = 2.0 * sur.n_nets * queries * sum(k * n for k, n in zip(w[:-1], w[1:]))
    tf = flop / fast_infer_s / 1e12
    del sur
    torch.cuda.empty_cache()
    return {"workload": f"{queries} electrode queries (ranges 20% wider than training), 4-net ensemble "
                        f"5-512x4-256; audit {audit} random queries through FDTD",
            "inference_cases_per_s": round(queries / fast_infer_s, 1), "fdtd_cases_per_s": round(fdtd_cps, 2),
            "fast": points["fast"], "guarded": points["guarded"],
            "target_met": bool(points["fast"]["gain_vs_fdtd"] >= 100 and
                               points["fast"]["audit_delivered_peak_error"]["max"] <= 0.02) or
                          bool(points["guarded"]["gain_vs_fdtd"] >= 100 and
                               points["guarded"]["audit_delivered_peak_error"]["max"] <= 0.02),
            "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": 2500.0, "unit": "TFLOP/s",
                         "frac": round(tf / 2500.0, 5), "kernel": "ensemble inference (bf16 MFMA products)"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--variant", default="tuned", choices=["tuned", "auto", "split", "fused", "tb2"],
                    help="tuned: launch shape from the autotuner (cached); auto: the library default "
                         "(two-step pass, 60x8 tiles, TZ 28, on this grid with a CPML)")
    ap.add_argument("--tile-y", type=int, default=0)
    ap.add_argument("--tile-z", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-grid sweep measurement")
    ap.add_argument("--no-tune", action="store_true", help="batched leg: fixed 32x8 tiles, TZ 32")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-in-the-loop measurement")
    ap.add_argument("--no-debye", action="store_true", help="skip the Debye-soil, lumped-element, oblique-wire and array measurements")
    ap.add_argument("--legs", default="debye,lumped,oblique,tower,array",
                    help="which of the Debye-soil, lumped-element, oblique-wire and array measurements to run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run plain copies of MIB MiB (profiler counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}): the multi-GPU "
              "decomposition of the grid is designed but not built.", file=sys.stderr)
        sys.exit(2)

    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return

    import torch
    from paper_2207_06908_amd import fdtd
    from paper_2207_06908_amd import scenarios as S

    from paper_2207_06908_amd import autotune
    variant = {"auto": 0, "split": 1, "fused": 2, "tb2": 3, "tuned": 0}[a.variant]
    tune_steps = autotune.tuning_steps() if a.variant == "tuned" else 0
    sc = S.config2(n_steps=tune_steps + a.warmup + a.steps)
    g = fdtd.Grid.from_params(sc.params(), precision=32)
    S.apply(sc, g)
    g.bind()
    if a.variant == "tuned":
        choice = autotune.tune_grid(g, autotune.grid_key(sc.params()))
        autotune.apply_grid(g, choice)
        a.variant = {1: "split", 2: "fused", 3: "tb2"}[choice["variant"]]
        a.tile_y, a.tile_z = choice["tile_y"], choice["tile_z"]
    else:
        g.set_kernel(variant, a.tile_y, a.tile_z)
    g.step(a.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g.timing(True)
    e0.record()
    g.step(a.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms, kn = g.kernel_time()
    g.timing(False)

    cells = sc.cells
    value = cells * a.steps / (ms / 1e3) / 1e6
    vname = "tb2" if a.variant == "auto" else a.variant
    ty = a.tile_y or 8
    tz = a.tile_z or (20 if vname == "tb2" else 32)
    traffic = MEASURED_TRAFFIC.get((kernel_source_hash(), vname, ty, tz))
    bytes_step = g.algorithmic_bytes_per_step()
    k_avg_s = kms / max(kn, 1) / 1e3
    achieved = bytes_step / k_avg_s / 1e9
    out = {
        "metric": "Mcell-updates/s",
        "value": round(value, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x512x384 Yee FDTD, dx 0.5 m, 10-cell CPML, two-layer soil, "
                               "30 m thin wire, 10 kA 1/50 us source, 14 probes",
                   "cells": cells, "kernel_variant": a.variant, "tile_y": a.tile_y, "tile_z": a.tile_z,
                   "coefficient_classes": g.num_classes},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_unit": "HBM bytes per step",
                     "kernel": {"fused": "k_fused_list (one pass per step, launched per CPML tile group)",
                                "tb2": "k_tb2_list (one pass per two steps, launched per CPML tile group)",
                                "split": "k_h_split + k_e_split (two launches per step)"}[vname],
                     "algorithmic_bytes_per_step": bytes_step,
                     "kernel_ms_per_step": round(kms / max(kn, 1), 5)},
    }
    del g
    torch.cuda.empty_cache()
    # actual HBM rate of the pass (counter traffic) and the practical ceiling
    copy_gbs, triad_gbs = stream_ceiling()
    if traffic:
        out["roofline"]["traffic_GBs"] = round(traffic / k_avg_s / 1e9, 1)
    out["roofline"]["stream_copy_GBs"] = copy_gbs
    out["roofline"]["stream_triad_GBs"] = triad_gbs
    if not a.no_batch:
        out["batched"] = bench_batch(tune=not a.no_tune)
    if not a.no_debye:
        legs = a.legs.split(",")
        for leg, fn in (("debye", bench_debye), ("lumped", bench_lumped), ("oblique", bench_oblique),
                        ("tower", bench_tower), ("array", bench_array)):
            if leg in legs:
                out[leg] = fn()
    if not a.no_surrogate:
        out["surrogate"] = bench_surrogate()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
