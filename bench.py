"""Benchmark of the LELBM time step on one MI355X.

Workload: the 2D four-quadrant Riemann input (1024 x 1024 periodic, seeded
states with density U[0.1,1.5], pressure U[0.03,1.5], velocity U[-1.2,1.2]
times the local sound speed, 1% smooth Fourier density perturbation).  One
step = one pass of the whole per-cell path (collision, stencil, entropic
reconstruction) and the moment-streaming gather over all cells.

Prints ONE JSON line (rank 0): MLUPS of the timed steps with inputs resident
in HBM, per-kernel durations measured with HIP events on the library's stream,
the roofline of the dominant kernel, and the CPU oracle's MLUPS on a bounded
sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--seed S]
                       [--n 1024] [--precision fp64|mixed] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "MLUPS per LELBM step: FP32+learned-EPR vs plain FP64, at matched L1 error"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# Algorithmic FP64 work of one stencil point in one reconstruction pass (2D):
# 27 monomial products (degree <= 6), 16 multiply-adds for the two exponents,
# 43 multiply-adds into the fluon (28) and phonon (15) moment sums, and two
# exponentials counted as 20 flops each (a degree-10 polynomial).
FLOPS_PER_POINT_PASS_2D = 27 + 2 * 16 + 2 * 43 + 2 * 20
# Algorithmic bytes of the gather: per arriving stencil point the (w_f, w_g)
# pair, per destination the written moments, per source its descriptor
# (velocity and radius).
GATHER_BYTES_PER_ARRIVAL = {"fp64": 16, "mixed": 8}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-window", type=int, default=256)
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (HBM counter calibration)")
    return ap.parse_args()


def cpu_baseline(cfg, prim, window, steps):
    """The oracle as it stands on a centred window of the same input (all four
    quadrant states, in equal parts), with no sources outside the window."""
    import oracle
    n = cfg["nx"]
    c = n // 2
    sl = slice(c - window // 2, c + window // 2)
    sub = {k: v[sl, sl] for k, v in prim.items()}
    wc = dict(cfg)
    wc.update(nx=window, ny=window, bc=["outflow"] * 4, pad=0)
    m = oracle.moments_from_primitives(2, wc["K"], sub["rho"], sub["ux"], sub["uy"], sub["RT"])
    t0 = time.perf_counter()
    st, out, stats, done = oracle.step(wc, m, steps)
    el = time.perf_counter() - t0
    if st != 0:
        raise RuntimeError("oracle failed on the CPU sample (%d)" % st)
    return {"value": window * window * steps / el / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%dx%d centre window of the same input, %d steps, no sources outside the window (%.1f s)"
                      % (window, window, steps, el)}


def main():
    a = parse()
    if a.copy_probe:
        import torch
        n = a.copy_probe // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}))
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the path has no multi-GPU decomposition "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import lelbm_inputs as li
    import paper_2508_06911_amd as lb

    torch.cuda.set_device(0)
    cfg, prim = li.quadrants(a.seed, n=a.n)
    prec = lb.FP64 if a.precision == "fp64" else lb.MIXED
    m = lb.moments_from_primitives(2, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
    stream = torch.cuda.current_stream()
    ctx = lb.Lelbm(cfg, m, precision=prec, stream=stream)
    if a.warmup:
        ctx.step(a.warmup)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    st = ctx.step(a.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    kt = ctx.kernel_times()
    persistent, scratch = ctx.memory()
    ctx.close()
    ncell = cfg["nx"] * cfg["ny"]
    mlups = ncell * a.steps / (ms * 1e-3) / 1e6

    epr_ms = kt["epr"][0] / max(kt["epr"][1], 1)
    gat_ms = kt["gather"][0] / max(kt["gather"][1], 1)
    flops = st["point_passes"] / a.steps * FLOPS_PER_POINT_PASS_2D
    epr_tflops = flops / (epr_ms * 1e-3) / 1e12
    esz = 8 if a.precision == "fp64" else 4
    gbytes = (st["arrivals"] / a.steps * GATHER_BYTES_PER_ARRIVAL[a.precision]
              + ncell * (11 * esz + 20))
    gat_gbs = gbytes / (gat_ms * 1e-3) / 1e9

    res = {
        "metric": METRIC,
        "value": round(mlups, 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms / a.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "2D four-quadrant Riemann input, %dx%d periodic, seed %d, %s path, "
                               "equilibrium Newton guess" % (a.n, a.n, a.seed, a.precision),
                   "cells": ncell, "steps_after_warmup": a.steps},
        "roofline": {"bound": "alu", "kernel": "k_epr (collision + stencil + Newton reconstruction)",
                     "achieved": round(epr_tflops, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(epr_tflops / FP64_PEAK_TFLOPS, 4), "traffic": None,
                     "avg_ms": round(epr_ms, 4),
                     "flops_per_launch": flops},
        "ms_gather": {"bound": "hbm", "kernel": "k_gather", "achieved": round(gat_gbs, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(gat_gbs / HBM_PEAK_GBS, 4), "avg_ms": round(gat_ms, 4),
                      "bytes_per_launch": gbytes},
        "kernels_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items() if v[1]},
        "newton_it": {"mean_f": round(st["it_mean_f"], 3), "max_f": st["it_max_f"],
                      "mean_g": round(st["it_mean_g"], 3), "max_g": st["it_max_g"]},
        "stencil_q": {"min": st["q_min"], "mean": round(st["q_mean"], 1), "max": st["q_max"]},
        "hbm_bytes": {"persistent": persistent, "scratch": scratch},
    }
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(cfg, prim, a.cpu_window, a.cpu_steps)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
