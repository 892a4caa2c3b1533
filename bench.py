"""Benchmark of the opacity + k-distribution hot path on one MI355X.

A step is one pass of the whole path over the mid-scale binary64 workload
(1e6 synthetic lines over 0-30000 cm^-1, 0.01 cm^-1 grid of 3e6 points,
100 cm^-1 cutoff, T = 1500 K, P = 1 atm, 300 bins x 20 Gauss-Legendre g):
per-line scaling and windows, the Voigt evaluation and accumulation kernel,
and the per-bin sort and k(g).  The line list is resident on the device
before timing starts.  Beside the headline the line reports the binary32
variant of the same step, the Chebyshev resampling and transmission of the
same bins, the batched tables (the same lines over 200 (T, P) states) and
the learned surrogate (1e8 lines, 25 cm^-1 cutoff, against the binary64
path) and a 1e7-line list streamed from host memory in 34 pieces.  Prints
one JSON line.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-f32]
                    [--no-resample] [--no-tables] [--no-surrogate] [--no-stream]
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "lines1e6_grid3e6"
PEAK_FP64_TFLOPS = 78.6  # MI355X binary64 vector peak
# Algorithmic work per line-point evaluation, by region, in the scope
# table's count: 7 operations common to every evaluation (offset, scaling,
# square, radius, region compare, line strength, accumulation), then for the
# 1-node rule one reciprocal (8); for the 3-node rule ~9 operations and 3
# reciprocals (19); for the series (2 ceil(x) + 14) terms of ~10 operations
# and a reciprocal each -- 24 terms on average over the series region -- plus
# erfcx, sin/cos and the two exponentials of the set-up (7 + 24 * 11 + 6 = 277).
FLOPS_PER_EVAL = {"gh1": 8, "gh3": 19, "core": 277}
DOMINANT_KERNEL = "wing_f64_kernel"
PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
# LDS rate assumed for the sort: 32 banks x 4 B per clock per CU, 256 CUs,
# 2.4 GHz
PEAK_LDS_GBS = 256 * 128 * 2.4
# surrogate training recipe: (Adam steps, learning rate) phases, batch 4096
SURROGATE_SCHEDULE = ((20000, 5e-3), (20000, 1e-3), (20000, 2e-4))
SURROGATE_WSCALE = 5.0  # loss weight 1/(1 + (z/5)^2)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "wing_f64_lines1e6_grid3e6_traffic.txt")
# what the dominant kernel's traffic depends on: its code, its line records
# and the order of its work items
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1503_03806_amd", "csrc", f)
                  for f in ("opacity_f64.hip", "hk_internal.h", "work_plan.hip", "line_prep.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel (fetch + write) from the
    committed counter summary, or None if the kernel's sources changed since
    the counters were taken."""
    try:
        kv = dict(line.split(":", 1) for line in open(TRAFFIC_FILE)
                  if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("kernel_sources_sha256_16") != kernel_digest():
        return None
    try:
        return int(kv["fetch_bytes_per_launch"]) + int(kv["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def synth_conditions(T, P):
    import synth
    return synth.conditions(T, P)


def cpu_baseline(w, points: int, one_thread_bins: int, kappa_gpu=None, k_gpu=None, f32=None, tables=None):
    """The oracle, built -O3 -march=native on this host, timed on all host
    threads over `points` grid points (whole bins, centred; the whole grid
    by default) and on one thread over `one_thread_bins` bins, opacity +
    k(g) each.  With the GPU's binary64 grid and k(g) table (host arrays),
    also their error against the oracle's: max and p99.9 per bin for kappa,
    max per bin for k(g); likewise, summarised, for the binary32 step's
    (f32 = (kappa, k(g))).  With the batched tables' k(g) (tables =
    (workload, array [state][bin][g])), their error against the oracle's on
    16 (state, bin) pairs drawn with seed 3 and the table's two corners (the
    oracle given the lines that can reach each bin); untimed."""
    import tempfile

    import numpy as np

    import oracle
    tmpdir = tempfile.mkdtemp(prefix="oracle_native")
    oracle.use_native(os.path.join(tmpdir, "liboracle_native.so"))
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    N = grid["n_points"]
    ppb = w.points_per_bin
    g, _ = oracle.g_nodes(w.n_g)

    def run(n_pts):
        j0 = (max(N - n_pts, 0) // 2 // ppb) * ppb  # centred, whole bins
        j1 = min(j0 + n_pts, N)
        t0 = time.perf_counter()
        kap, evals = oracle.opacity(lines, cond, grid, j0, j1)
        kd = oracle.kdist(kap, ppb, g)
        return j0, j1, kap, kd, evals, time.perf_counter() - t0

    cores = oracle.num_threads()
    j0, j1, kap, kd, evals, dt = run(points)
    rec = {"value": evals / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
           "build": "gcc -O3 -march=native -ffp-contract=off, OpenMP static schedule",
           "sample": "grid points %d..%d (%d of %d bins) of %s, all %d lines: %d evals "
                     "in %.2f s, opacity + k(g)" % (j0, j1, (j1 - j0) // ppb, N // ppb,
                                                   w.name, len(lines["nu"]), evals, dt)}
    if kappa_gpu is not None and j0 == 0 and j1 == N:
        pos = kap > 0
        assert np.array_equal(pos, kappa_gpu > 0)
        e = np.zeros(N)
        e[pos] = np.abs(kappa_gpu[pos] / kap[pos] - 1.0)
        eb = e.reshape(-1, ppb)
        ek = np.abs(k_gpu / kd - 1.0).max(axis=1)

        def r3(a):
            return [float("%.3g" % v) for v in a]
        rec["error_vs_oracle"] = {
            "what": "relative error of the GPU binary64 step's results against the oracle's, per bin",
            "kappa_max": float(eb.max()), "kappa_p999_worst_bin": float(np.quantile(eb, 0.999, axis=1).max()),
            "kg_max": float(ek.max()), "bins": int(eb.shape[0]),
            "kappa_max_per_bin": r3(eb.max(axis=1)),
            "kappa_p999_per_bin": r3(np.quantile(eb, 0.999, axis=1)),
            "kg_max_per_bin": r3(ek)}
        if f32 is not None:
            k32, kd32 = f32
            assert np.array_equal(pos, k32 > 0)
            e = np.zeros(N)
            e[pos] = np.abs(k32[pos] / kap[pos] - 1.0)
            eb = e.reshape(-1, ppb)
            rec["error_vs_oracle_f32"] = {
                "what": "relative error of the GPU binary32 + compensated step's results against the oracle's",
                "kappa_max": float(eb.max()),
                "kappa_p999_worst_bin": float(np.quantile(eb, 0.999, axis=1).max()),
                "kg_max": float(np.abs(kd32 / kd - 1.0).max()), "bins": int(eb.shape[0])}
    if tables is not None:
        tw, tab = tables
        t_lines, t_grid = tw.lines(), tw.grid()
        t_ppb = tw.points_per_bin
        tg, _ = oracle.g_nodes(tw.n_g)
        n_states, n_bins = tab.shape[0], tab.shape[1]
        rng = np.random.default_rng(3)
        pairs = [(0, 0), (n_states - 1, n_bins - 1)] + [
            (int(a), int(b)) for a, b in zip(rng.choice(n_states, 16, replace=False), rng.choice(n_bins, 16))]
        worst = 0.0
        for s_, b in pairs:
            T, P = tw.states[s_]
            c = synth_conditions(T, P)
            j0, j1 = b * t_ppb, min((b + 1) * t_ppb, t_grid["n_points"])
            lo = t_grid["nu_min"] + j0 * t_grid["dnu"] - t_grid["cutoff"] - 1.0
            hi = t_grid["nu_min"] + (j1 - 1) * t_grid["dnu"] + t_grid["cutoff"] + 1.0
            keep = (t_lines["nu"] >= lo) & (t_lines["nu"] <= hi)
            near = {k: v[keep] for k, v in t_lines.items() if v is not None}
            ref, _ = oracle.opacity(near, c, t_grid, j0, j1)
            kr, _ = oracle.kdist_bin(ref, tg)
            worst = max(worst, float(np.abs(tab[s_, b] / kr - 1.0).max()))
        rec["error_vs_oracle_tables"] = {
            "what": "max relative error of the batched binary32 tables' k(g) against the oracle's, "
                    "on 16 (state, bin) pairs drawn with seed 3 and the table's two corners",
            "kg_max": worst, "pairs": len(pairs)}
    oracle.set_num_threads(1)
    j0, j1, _, _, evals1, dt1 = run(one_thread_bins * ppb)
    oracle.set_num_threads(cores)
    rec["one_thread"] = {"value": evals1 / dt1, "unit": "evals/s", "cores": 1,
                         "sample": "grid points %d..%d (%d bins): %d evals in %.2f s, opacity + k(g)"
                                   % (j0, j1, (j1 - j0) // ppb, evals1, dt1)}
    return rec


def bench_resample(hk, torch, ctx, kappa, N, ppb, g):
    """Steps after k(g) on the headline grid (last binary64 opacity): sort
    with the sorted bins kept, 20 Chebyshev coefficients per bin, and the
    transmission for 1000 column masses per bin."""
    import numpy as np
    sorted_k = torch.empty_like(kappa)
    m_col = torch.tensor(np.logspace(-18.0, 30.0, 1000), device="cuda")
    def once():
        ctx.kdist(kappa, ppb, g, sorted_out=sorted_k)
        coef = ctx.resample(sorted_k, ppb, 20)
        return ctx.transmission(coef, m_col)
    once()
    torch.cuda.synchronize()
    reps = 5
    gc.collect()
    t0 = time.perf_counter()
    for _ in range(reps):
        once()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    t1 = time.perf_counter()
    coef = ctx.resample(sorted_k, ppb, 20)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t1
    t1 = time.perf_counter()
    ctx.transmission(coef, m_col)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t1
    return {"bins": int(-(-N // ppb)), "n_coef": 20, "n_m": 1000,
            "ms_sort_fit_transmission": 1e3 * dt, "ms_fit": 1e3 * t_fit, "ms_transmission": 1e3 * t_tr}


def kdist_stage(ms, N, ppb, n_g, key_bytes=8, radix_max_keys=16384):
    """The Sort + k(g) stage against HBM and LDS: its algorithmic bytes (each
    opacity read once, k(g) written once) and the LDS traffic of the
    per-bin radix sort (bins of up to 16384 keys, one workgroup each): every
    pass (8 bits of the key) writes each key to its place and reads it back;
    binary64 keys take the 4 passes of their high words, then a finish of the
    runs of equal high words (the full 8 passes only when a run is long)."""
    n_bins = -(-N // ppb)
    hbm = key_bytes * N + 8 * n_bins * n_g
    out = {"ms": ms, "hbm_bytes": hbm, "GB_s": hbm / (ms * 1e-3) / 1e9,
           "frac_of_hbm_peak": hbm / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    if ppb <= radix_max_keys:
        passes = 4
        lds = passes * 2 * key_bytes * N
        out.update({"sort": "LDS radix, one workgroup per bin", "passes": passes,
                    "lds_bytes": lds, "lds_GB_s": lds / (ms * 1e-3) / 1e9,
                    "frac_of_lds_peak": lds / (ms * 1e-3) / 1e9 / PEAK_LDS_GBS,
                    "bound": "VALU work of the ballot ranking per CU, and the tail of 300 workgroups "
                             "on 256 CUs"})
    return out


def bench_stream(hk, torch, ctx, n_chunks: int = 34):
    """A list streamed from host memory: the 1e7-line binary32 workload cut
    into 34 wavenumber-ordered pieces (the paper's largest list came in 34
    files), timed wall-clock from host arrays to the finished grid, against
    the same opacity call on the list already resident on the device and
    against loading and accumulating the pieces one call at a time."""
    import numpy as np
    import synth
    w = synth.WORKLOADS["lines1e7_fp32"]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    log("bench: stream, %d lines in %d chunks" % (len(lines["nu"]), n_chunks))
    order = np.argsort(lines["nu"], kind="stable")
    ordered = {k: np.ascontiguousarray(v[order]) for k, v in lines.items()}
    cuts = np.linspace(0, len(order), n_chunks + 1).astype(int)
    chunks = [{k: v[a:b] for k, v in ordered.items()} for a, b in zip(cuts[:-1], cuts[1:])]
    prec = hk.HK_F32_KAHAN
    out = torch.empty(grid["n_points"], dtype=torch.float64, device="cuda")

    def wall(fn, reps, warm=1):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        # a full collection of Python's cyclic garbage collector, which
        # otherwise falls every few calls into the marshalling of the 34
        # pieces' arguments (~40-60 ms on the host, none of it the library's)
        gc.collect()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / reps

    ms_stream = wall(lambda: ctx.opacity_stream(chunks, cond["mass_amu"], st, grid, prec, out=out,
                                                T_ref=cond["T0"]), 3)
    evals = ctx.stats()["evals"]

    def sequential():
        for i, c in enumerate(chunks):
            ctx.load_lines(c, cond["mass_amu"], cond["T0"])
            ctx.opacity(st, grid, prec, out=out, accumulate=i > 0)
    ms_seq = wall(sequential, 1)
    t0 = time.perf_counter()
    ctx.load_lines(ordered, cond["mass_amu"], cond["T0"])
    ms_load = 1e3 * (time.perf_counter() - t0)
    ms_res = wall(lambda: ctx.opacity(st, grid, prec, out=out), 3)
    return {"workload": w.name, "chunks": n_chunks, "precision": "f32_kahan", "evals": evals,
            "ms_streamed": ms_stream, "ms_resident_opacity": ms_res,
            "ms_load_whole_list": ms_load, "ms_load_and_opacity_per_chunk": ms_seq,
            "host_bytes": 8 * 5 * len(order),
            "streamed_over_resident": ms_stream / ms_res}


def bench_tables(hk, torch, ctx, g):
    """The batched tables: the same 1e6 lines over 20 x 10 (T, P) states,
    binary32 profiles, k(g) for 300 bins x 20 g per state; one untimed call
    (it times the tile shapes once), then one timed call."""
    import synth
    w = synth.WORKLOADS["lines1e6_tables200"]
    grid = w.grid()
    states = [{k: c[k] for k in ("T", "P", "P_self", "q_ratio")}
              for c in (synth.conditions(T, P) for T, P in w.states)]
    log("bench: tables, %d states" % len(states))
    out = torch.empty((len(states), w.n_bins, w.n_g), dtype=torch.float64, device="cuda")
    ctx.tables(states, grid, w.points_per_bin, g, hk.HK_F32_KAHAN, out=out)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    gc.collect()
    t0 = time.perf_counter()
    ctx.tables(states, grid, w.points_per_bin, g, hk.HK_F32_KAHAN, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tm = ctx.timing()
    ctx.set_timing(False)
    evals = ctx.stats()["evals"]
    return ({"workload": w.name, "states": len(states), "precision": "f32_kahan",
             "value": evals / dt, "unit": "evals/s", "ms_per_call": 1e3 * dt, "evals": evals,
             "points_per_lane": ctx.get_option("tables_points_per_lane"),
             "stage_ms": {k: v[0] for k, v in tm.items()}}, (w, out.cpu().numpy()))


def bench_surrogate(hk, torch, ctx, n_lines: int = 0, train_steps: int = 0):
    """The learned surrogate: trained on 1e7 samples (x in [0, 50], y in
    [1e-4, 1e2], targets from the plain method), certified at a 2e-5
    per-evaluation budget, then the opacity of 1e8 lines (0.01 cm^-1 grid of
    3e6 points, 25 cm^-1 cutoff, 1500 K, 1 atm) with the surrogate, with the
    binary32 path and with the binary64 path; error against binary64."""
    import synth
    w = synth.WORKLOADS["lines1e8_surrogate"]
    if n_lines:
        import dataclasses
        w = dataclasses.replace(w, n_lines=n_lines)
    schedule = SURROGATE_SCHEDULE
    if train_steps:
        total = sum(s for s, _ in schedule)
        schedule = tuple((max(1, s * train_steps // total), lr) for s, lr in schedule)
    log("bench: surrogate training")
    x, y = synth.surrogate_samples(10_000_000, seed=7)
    xd = torch.tensor(x, device="cuda")
    yd = torch.tensor(y, device="cuda")
    zd = ctx.surrogate_labels(xd, yd)
    ctx.surrogate_set_params(synth.mlp_init(7))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = []
    for steps, lr in schedule:
        hist.append(ctx.surrogate_train(xd, yd, zd, batch=4096, steps=steps, lr=lr,
                                        wscale=SURROGATE_WSCALE))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    hist = torch.cat(hist).cpu()
    err, count = ctx.surrogate_certify(2e-5)
    del xd, yd, zd
    log("bench: surrogate workload, generating %d lines" % w.n_lines)
    lines, cond = w.lines(), w.conditions()
    grid = w.grid()
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    del lines
    st = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    res = {}
    for name, prec in (("f64", hk.HK_F64), ("f32_kahan", hk.HK_F32_KAHAN),
                       ("f32_surrogate", hk.HK_F32_SURROGATE)):
        k = ctx.opacity(st, grid, prec)
        torch.cuda.synchronize()
        ctx.set_timing(True)
        gc.collect()
        t0 = time.perf_counter()
        for _ in range(2):
            ctx.opacity(st, grid, prec, out=k)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 2
        tm = ctx.timing()
        ctx.set_timing(False)
        res[name] = (k, dt, {kk: v[0] / max(v[1], 1) for kk, v in tm.items()}, ctx.stats())
    evals = ctx.stats()["evals"]
    ref = res["f64"][0]
    out = {"workload": w.name if not n_lines else "%s (%d lines)" % (w.name, n_lines),
           "n_lines": w.n_lines, "evals": evals,
           "train_samples": 10_000_000, "train_steps": int(len(hist)), "train_s": train_s,
           "loss_first": float(hist[0]), "loss_last100": float(hist[-100:].mean()),
           "certified_cells": count, "cells": int(err.size), "budget": 2e-5}
    for name, (k, dt, stage, stt) in res.items():
        pos = ref > 0
        out[name] = {"ms": 1e3 * dt, "evals_per_s": evals / dt, "stage_ms": stage,
                     "max_rel_err_vs_f64": float(((k[pos] - ref[pos]).abs() / ref[pos]).max())}
        if name == "f32_surrogate":
            out[name]["evals_surrogate"] = stt["evals_surrogate"]
            out[name]["network_share_of_series_region"] = stt["evals_surrogate"] / max(stt["evals_core"], 1)
    out["series_kernel_ms"] = {"f32_kahan": res["f32_kahan"][2]["core"],
                               "f32_surrogate": res["f32_surrogate"][2]["core"]}
    out["speedup_surrogate_vs_f64"] = res["f64"][1] / res["f32_surrogate"][1]
    out["speedup_surrogate_vs_f32"] = res["f32_kahan"][1] / res["f32_surrogate"][1]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true", help="skip the binary32 variant")
    ap.add_argument("--no-tables", action="store_true", help="skip the batched tables")
    ap.add_argument("--no-resample", action="store_true",
                    help="skip the Chebyshev resampling + transmission leg")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate workload")
    ap.add_argument("--no-stream", action="store_true", help="skip the streamed line list")
    ap.add_argument("--surrogate-lines", type=int, default=0,
                    help="lines of the surrogate leg (default: the workload's 1e8; fewer for profiling)")
    ap.add_argument("--surrogate-train-steps", type=int, default=0,
                    help="Adam steps of the surrogate training (default: the full recipe)")
    ap.add_argument("--cpu-points", type=int, default=3000000,
                    help="grid points in the oracle's timed sample (all threads)")
    ap.add_argument("--cpu-one-thread-bins", type=int, default=8,
                    help="bins in the oracle's one-thread timed sample")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this size (counter "
                         "calibration)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(got --gpus %d)" % a.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_1503_03806_amd as hk
    import synth

    w = synth.WORKLOADS[WORKLOAD]
    lines, cond, grid = w.lines(), w.conditions(), w.grid()
    state = {k: cond[k] for k in ("T", "P", "P_self", "q_ratio")}
    N, ppb = grid["n_points"], w.points_per_bin
    n_bins = -(-N // ppb)
    log("bench: %s, %d lines, %d points" % (w.name, len(lines["nu"]), N))

    ctx = hk.Context(0)
    ctx.load_lines(lines, cond["mass_amu"], cond["T0"])
    g, _ = hk.hk_gauss_legendre(w.n_g)
    kappa = torch.empty(N, dtype=torch.float64, device="cuda")
    k_out = torch.empty((n_bins, w.n_g), dtype=torch.float64, device="cuda")

    def timed(precision, steps):
        def step():
            hk.hk_opacity(ctx.h, state, grid, precision, kappa)
            hk.hk_kdist(ctx.h, kappa, hk.HK_F64, N, ppb, g, k_out)
        for _ in range(a.warmup):
            step()
        torch.cuda.synchronize()
        ctx.set_timing(True)
        gc.collect()  # no collection of Python's garbage collector in the timed steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        tm = ctx.timing()
        ctx.set_timing(False)
        return elapsed, tm

    # the binary32 + compensated-sum variant of the same step, reported beside
    # the binary64 headline (its result differs from binary64 by ~1e-6)
    f32_elapsed, f32_tm, f32_host = (None, None, None)
    if not a.no_f32:
        f32_elapsed, f32_tm = timed(hk.HK_F32_KAHAN, max(1, a.steps // 2))
        f32_host = (kappa.cpu().numpy(), k_out.cpu().numpy())
    elapsed, tm = timed(hk.HK_F64, a.steps)
    st = ctx.stats()
    kappa_host, k_host = kappa.cpu().numpy(), k_out.cpu().numpy()  # for the error against the oracle
    if a.calib_copy_mib:
        n = a.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (8 * n, 8 * n))

    evals = st["evals"]
    ms_step = 1e3 * elapsed / a.steps
    # the dominant kernel: the Gauss-Hermite wing kernel (stage "opacity")
    op_ms = tm["opacity"][0] / max(tm["opacity"][1], 1)
    flops = FLOPS_PER_EVAL["gh1"] * st["evals_gh1"] + FLOPS_PER_EVAL["gh3"] * st["evals_gh3"]
    achieved = flops / (op_ms * 1e-3) / 1e12
    step_flops = flops + FLOPS_PER_EVAL["core"] * st["evals_core"]
    # the wing's algorithmic bytes: each line record (64 B) read once, each
    # grid value (8 B) written once
    alg_bytes = 64 * len(lines["nu"]) + 8 * N
    traffic = measured_traffic()
    rec = {
        "metric": "Voigt line-point evals/s (opacity + k(g) wall time per step in ms_per_step)",
        "value": evals * a.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n_lines": len(lines["nu"]), "n_points": N,
                   "dnu": grid["dnu"], "cutoff": grid["cutoff"], "T": cond["T"],
                   "P_atm": cond["P"], "n_bins": n_bins, "n_g": w.n_g, "precision": "f64",
                   "evals_per_step": evals, "evals_core": st["evals_core"],
                   "evals_gh3": st["evals_gh3"], "evals_gh1": st["evals_gh1"]},
        "stage_ms": {k: v[0] / max(v[1], 1) for k, v in tm.items()},
        "kdist": kdist_stage(tm["kdist"][0] / max(tm["kdist"][1], 1), N, ppb, w.n_g),
        "stage_note": "event-timed mean per timed launch; 'opacity' (wing) and 'core' (series) run concurrently "
                      "on two streams and overlap; 'line_prep' includes tile ranges and work plans",
        "roofline": {"bound": "alu", "kernel": DOMINANT_KERNEL,
                     "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "flops_per_launch": flops, "launch_ms": op_ms,
                     "flops_per_eval": FLOPS_PER_EVAL,
                     "algorithmic_bytes": alg_bytes,
                     "traffic_over_algorithmic": (traffic / alg_bytes) if traffic else None,
                     "concurrent_with": "core_f64_kernel on a second stream (launch_ms includes "
                                        "the time the two share the device)",
                     "step": {"flops": step_flops, "achieved": step_flops / (ms_step * 1e-3) / 1e12,
                              "frac": step_flops / (ms_step * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                              "what": "wing + series algorithmic work over the whole step's wall time"}},
    }
    if f32_tm is not None:
        f32_steps = max(1, a.steps // 2)
        rec["f32_kahan"] = {
            "value": evals * f32_steps / f32_elapsed, "unit": "evals/s",
            "ms_per_step": 1e3 * f32_elapsed / f32_steps,
            "stage_ms": {k: v[0] / max(v[1], 1) for k, v in f32_tm.items()},
            "speedup_vs_f64": (1e3 * elapsed / a.steps) / (1e3 * f32_elapsed / f32_steps)}
    if not a.no_resample:
        rec["resample"] = bench_resample(hk, torch, ctx, kappa, N, ppb, g)
    tables_host = None
    if not a.no_tables:
        rec["tables"], tables_host = bench_tables(hk, torch, ctx, g)
    if not a.no_stream:
        rec["stream"] = bench_stream(hk, torch, ctx)
    if not a.no_cpu_baseline:
        log("bench: timing the oracle on a sample")
        rec["cpu_baseline"] = cpu_baseline(w, a.cpu_points, a.cpu_one_thread_bins, kappa_host, k_host,
                                           f32_host, tables_host)
        if "error_vs_oracle" in rec["cpu_baseline"]:
            rec["error_vs_oracle"] = rec["cpu_baseline"].pop("error_vs_oracle")
        if "error_vs_oracle_f32" in rec["cpu_baseline"] and "f32_kahan" in rec:
            rec["f32_kahan"]["error_vs_oracle"] = rec["cpu_baseline"].pop("error_vs_oracle_f32")
        if "error_vs_oracle_tables" in rec["cpu_baseline"] and "tables" in rec:
            rec["tables"]["error_vs_oracle"] = rec["cpu_baseline"].pop("error_vs_oracle_tables")
    if not a.no_surrogate:
        rec["surrogate"] = bench_surrogate(hk, torch, ctx, a.surrogate_lines, a.surrogate_train_steps)
    ctx.close()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
