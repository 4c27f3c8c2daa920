"""Benchmark of the LELBM time step on one MI355X.

Workload: the 2D four-quadrant Riemann input, 2048 x 2048 periodic (seeded
states with density U[0.1,1.5], pressure U[0.03,1.5], velocity U[-1.2,1.2]
times the local sound speed, 1% smooth Fourier density perturbation).  One
step = one pass of the whole per-cell path (collision, stencil, entropic
reconstruction) and the moment-streaming gather over all cells.

Protocol:
  1. harvest (features -> converged multipliers) pairs from plain FP64 runs of
     the 1024 x 1024 input on other seeds;
  2. train the warm-start network on them with the library's own kernels;
  3. run the 2048 x 2048 input from the same initial state with
       fp64-eq   plain FP64 path, equilibrium (IID13) Newton guess,
       mixed-mlp FP32 records (FP64 state and sums) + learned Newton guess,
     and, for attribution, the other combinations of {fp64, mixed} with
     {eq, mlp, lin (closed-form linearised guess), prev (linearised guess
     plus the previous step's correction)}, W untimed warmup steps then K
     timed steps each, inputs resident in HBM;
  4. L1 errors of density, velocity and temperature of every run against the
     fp64-eq run after the same steps.

Prints ONE JSON line: ``value`` = MLUPS of the mixed-mlp run; the FP64 MLUPS,
the errors, Newton iterations, per-kernel times (HIP events on the library's
stream), the roofline of the dominant kernel (the per-cell reconstruction
kernel), the gather's HBM fraction and the CPU oracle's MLUPS on a bounded
sample of the same workload.  Context runs (unless --no-context): the
paper's hot box at RT 0.5 and 2 (4096 x 4096), the 4096 x 2048 channel and
the 8192 x 4096 Mach-10 channel (unless --no-c4), FP64 and FP32 from one
developed state with per-field L1 errors.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--seed S] [--n 2048]
                       [--runs fp64-eq,mixed-mlp,...] [--no-cpu] [--no-context]
"""
import argparse
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "MLUPS per LELBM step: FP32+learned-EPR vs plain FP64, at matched L1 error"
HBM_PEAK_GBS = 8000.0
# MI355X vector peak: 256 CUs x 64 lanes x 2.4 GHz x 2 (FMA).  FP64 and
# non-packed FP32 run at the same rate; packed FP32 math is disabled in this
# build, so the same figure bounds both paths.
VALU_PEAK_TFLOPS = 78.6
# FP64 work of the reconstruction kernel as written.  The stencil points'
# exponentials come from product recurrences along the rows and down the
# first column (exact exponentials only at a few starts per row and pass), so
# the count follows the code rather than the method's one-exponential-per-
# point cost model:
#   33 per point and Newton evaluation: x^2..x^6 (5 multiplies + the offset),
#      12 moment-sum updates (10 of them multiply-adds), 5 recurrence products
#    7 per point of the final pass: two weights, five recurrence products
#  100 per stencil row and pass: folding the row sums into the 28 + 15
#      monomial sums (43 multiply-adds), y powers, the column recurrence
# 1480 per evaluation: Hessian assembly, Cholesky factorisations of the
#      10x10 and 6x6 systems and their solves (~1100), the column's and the
#      recurrence ratios' exponentials (16 at ~20 flops each, plus setup)
#  630 per cell: collision, linearised guess, the final pass's exponentials
# (the learned guess's 12.3 kFLOP per cell run on MFMA in BF16 and are not
# counted against the FP64 peak).
FLOPS_POINT_EVAL, FLOPS_POINT_FINAL, FLOPS_ROW, FLOPS_EVAL, FLOPS_CELL = 33, 7, 100, 1480, 630


def epr_flops_per_step(st, steps):
    """Executed FP64 flops of the reconstruction kernels per step from the
    step statistics (sums over cells and steps): point_passes = sum of
    q x passes, q_mean x cells = sum of q, row_passes = sum of rows x passes;
    cells with refined stencils (a separate point-by-point kernel) are left
    out of the point terms.  The evaluations per cell are passes - 1, their
    sum taken as point_passes / q_mean - cells."""
    pp = st["point_passes"] - st["point_passes_refined"]
    q = st["q_mean"] * st["cells"]
    eval_points = max(pp - q, 0.0)
    evals = max(pp / max(st["q_mean"], 1e-30) - st["cells"], 0.0)
    return (FLOPS_POINT_EVAL * eval_points + FLOPS_POINT_FINAL * q + FLOPS_ROW * st["row_passes"]
            + FLOPS_EVAL * evals + FLOPS_CELL * st["cells"]) / steps


# FP64 work of the 3D reconstruction kernel (k3_epr) as written, per unit
# (a multiply-add counts 2):
#   28 per point and Newton evaluation: x, the five product recurrences, x^1..x^6
#      and x^1..x^4 (10 multiplies) and 12 row-sum updates
#    8 per point of the final pass: x, the recurrences, two weights
#  330 per stencil row and pass: the exponents' row coefficients (29 terms), y
#      powers, folding the row sums into the 28 + 15 plane sums, and the
#      recurrences' start values (their polynomials and five exponentials of ~22)
#   50 per stencil row, once per cell: the row spans (the exact ball test at the
#      span ends), tabulated in LDS for all passes (the table covers the
#      (2R + 3)^2 rows of the box, about twice the rows that hold points)
#  250 per stencil plane and pass: z powers and folding the plane sums into
#      the 84 + 35 monomial sums; planes are not counted by the step
#      statistics and are taken as rows x 2 / (pi (R + 1/2)) (the planes and
#      rows of a ball), with R + 1/2 from the mean stencil size
# 6050 per evaluation: the 19x19 and 10x10 Hessians, their Cholesky
#      factorisations and solves, the two constant recurrence factors
#  300 per cell: collision
FLOPS3_POINT_EVAL, FLOPS3_POINT_FINAL, FLOPS3_ROW, FLOPS3_PLANE, FLOPS3_EVAL, FLOPS3_CELL = 28, 8, 330, 250, 6050, 300
FLOPS3_SPAN = 50


def epr3_flops_per_step(st, steps):
    """Executed FP64 flops of k3_epr per step from the step statistics."""
    q = st["q_mean"] * st["cells"]
    eval_points = max(st["point_passes"] - q, 0.0)
    evals = max(st["point_passes"] / max(st["q_mean"], 1e-30) - st["cells"], 0.0)
    radius = (3.0 * st["q_mean"] / (4.0 * math.pi)) ** (1.0 / 3.0)
    planes = st["row_passes"] * 2.0 / (math.pi * max(radius, 1.0))
    rows_once = st["row_passes"] / (evals / max(st["cells"], 1) + 1.0)    # passes = evaluations + the final pass
    return (FLOPS3_POINT_EVAL * eval_points + FLOPS3_POINT_FINAL * q + FLOPS3_ROW * st["row_passes"]
            + FLOPS3_PLANE * planes + FLOPS3_SPAN * rows_once + FLOPS3_EVAL * evals
            + FLOPS3_CELL * st["cells"]) / steps


# Algorithmic bytes of the gather: per arriving stencil point the (w_f, w_g)
# pair, per destination the written moments, per source its descriptor
# (velocity, density, temperature, radius: 20 bytes).
GATHER_PAIR_BYTES = {"fp64": 16, "mixed": 8}
GATHER_DESC_BYTES = 20
RUNS = ("fp64-eq", "mixed-mlp", "mixed-eq", "fp64-mlp", "mixed-lin", "fp64-lin", "mixed-prev", "fp64-prev",
        "mixed-mlpprev", "fp64-mlpprev")
# The paper's own timings (hot-box advection, 4096^2, RTX 4070), as context.
PAPER_HOTBOX_S_PER_STEP = {0.5: 10.9, 2.0: 33.8}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--runs", default=",".join(RUNS))
    ap.add_argument("--harvest-n", type=int, default=1024)
    ap.add_argument("--harvest-seeds", default="0,1,2,3")
    ap.add_argument("--harvest-steps", type=int, default=100)
    ap.add_argument("--harvest-pairs", type=int, default=10_000_000)
    ap.add_argument("--train-steps", type=int, default=12000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--scratch-budget", type=float, default=0,
                    help="population scratch budget in bytes (0: the library's default)")
    ap.add_argument("--cpu-window", type=int, default=512)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-context", action="store_true", help="skip the hot-box and channel context runs")
    ap.add_argument("--channel-seed", type=int, default=0)
    ap.add_argument("--channel-warmup", type=int, default=300)
    ap.add_argument("--channel-steps", type=int, default=10)
    ap.add_argument("--c4-warmup", type=int, default=200)
    ap.add_argument("--c4-steps", type=int, default=3)
    ap.add_argument("--no-c4", action="store_true", help="skip the 8192x4096 Mach-10 channel context run")
    ap.add_argument("--horizon-steps", type=int, default=2000,
                    help="steps of the 2048^2 four-quadrant and 4096x2048 channel horizon runs (0: skip)")
    ap.add_argument("--c4-horizon", type=int, default=0,
                    help="only run the 8192x4096 Mach-10 channel for this many steps on both paths "
                         "(FP64 and FP32 + learned guess) and report the L1 error per field")
    ap.add_argument("--c4-horizon-runs", default="fp64-eq,mixed-mlp",
                    help="the reference and the compared path of --c4-horizon (fp64-eq, fp64-lin, mixed-mlp, "
                         "mixed-eq)")
    ap.add_argument("--c4-horizon-seconds", type=float, default=900.0,
                    help="wall-time limit of the --c4-horizon run (it stops at the last whole chunk)")
    ap.add_argument("--channel-only", action="store_true",
                    help="run only the 4096x2048 channel context (for kernel traces of that workload)")
    ap.add_argument("--c4-only", action="store_true",
                    help="run only the 8192x4096 Mach-10 channel context, FP32 path with the learned guess "
                         "(for kernel traces of that workload)")
    ap.add_argument("--d3", type=int, default=0,
                    help="time the 3D step on an N^3 periodic box instead (its own JSON line)")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="only run a plain device copy of this many bytes (HBM counter calibration)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def primitives(mom, dim=2, K=3.0):
    """Density, velocity and RT from raw 2D moments [11][cells] (measurement
    only)."""
    rho = mom[0]
    ux, uy = mom[1] / rho, mom[2] / rho
    rt = ((mom[3] + mom[5] + mom[8]) / rho - ux * ux - uy * uy) / (dim + K)
    return rho, ux, uy, rt


def l1_errors(a, b):
    """Relative L1 errors of (rho, u, T) of moments a against reference b."""
    ra, uxa, uya, ta = primitives(a)
    rb, uxb, uyb, tb = primitives(b)
    return {
        "rho": float(np.abs(ra - rb).sum() / np.abs(rb).sum()),
        "u": float((np.abs(uxa - uxb) + np.abs(uya - uyb)).sum() / (np.abs(uxb) + np.abs(uyb)).sum()),
        "T": float(np.abs(ta - tb).sum() / np.abs(tb).sum()),
    }


KERNEL_SOURCES = {"2d": ("lelbm_kernels.hip", "lelbm_internal.h", "lelbm_mlp_dev.h"),
                  "3d": ("lelbm_3d.hip", "lelbm_3d.h", "lelbm_internal.h")}


def kernel_source_sha(dim="2d"):
    """sha256 over the sources compiled into the 2D (or 3D) kernels, in a fixed order."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[dim]:
        with open(os.path.join(ROOT, "paper_2508_06911_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(dim="2d"):
    """HBM traffic per launch from committed counter summaries: a line
    ``TRAFFIC {json}`` in profiles/*.md whose ``source_sha256`` equals the
    hash of the current sources of the 2D (or 3D) kernels (the kernel file
    and the headers it includes: any change to them voids the figure)."""
    sha = kernel_source_sha(dim)
    out = {}
    for p in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(p) as f:
            for line in f:
                m = re.match(r"^TRAFFIC (\{.*\})\s*$", line.strip())
                if m:
                    d = json.loads(m.group(1))
                    if d.get("source_sha256") == sha:
                        out[(d["kernel"], d["workload"])] = d["bytes_per_launch"]
    return out


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
    return {"value": round(window * window * steps / el / 1e6, 5), "unit": "MLUPS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%dx%d centre window of the same input, %d steps, no sources outside the window (%.1f s)"
                      % (window, window, steps, el)}


def harvest_and_train(a, lb, li, torch, prev=False):
    """Harvest (features, correction) pairs from FP64 runs of the four-quadrant
    input at the harvest size and train the network on them.  With prev the
    harvest runs use the previous-step guess, so the targets are what the
    network should add to it (for the learned + previous-step guess)."""
    seeds = [int(s) for s in a.harvest_seeds.split(",") if s]
    cells = a.harvest_n * a.harvest_n
    stride = max(1, (cells * a.harvest_steps * len(seeds)) // a.harvest_pairs)
    cap = a.harvest_pairs + cells // stride + 1
    buf = torch.zeros((cap, 32), dtype=torch.float32, device="cuda")
    t0 = time.perf_counter()
    n = 0
    for s in seeds:
        if n >= cap:
            break
        cfg, prim = li.quadrants(s, n=a.harvest_n)
        m = lb.moments_from_primitives(2, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
        c = lb.Lelbm(cfg, m, guess=lb.GUESS_PREV if prev else lb.GUESS_EQ)
        c.harvest(buf[n:], stride=stride)        # each context counts from 0
        c.step_nostats(a.harvest_steps)
        n = min(cap, n + c.harvest_count())
        c.close()
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t0
    log("harvested %d pairs (stride %d%s) in %.1f s" % (n, stride, ", previous-step guess" if prev else "", t_h))
    g = torch.Generator(device="cpu").manual_seed(1234)
    perm = torch.randperm(n, generator=g).to("cuda")
    nval = min(200_000, n // 20)
    val = buf[perm[:nval]].contiguous()
    train = buf[perm[nval:]].contiguous()
    del buf, perm
    mlp = lb.Mlp(seed=1)
    mlp.fit_normalization(train)
    t0 = time.perf_counter()
    # three phases of constant-rate Adam with decreasing step size
    phases = ((0.5, 2e-3), (0.3, 7e-4), (0.2, 2e-4))
    loss = None
    for i, (frac, lr) in enumerate(phases):
        loss = mlp.train(train, steps=max(1, int(a.train_steps * frac)), batch=a.batch, lr=lr, seed=7 + i)
    torch.cuda.synchronize()
    t_t = time.perf_counter() - t0
    _, vmse = mlp.gradient(val)
    log("trained %d steps in %.1f s: train loss %.4f, held-out mse %.4f" % (a.train_steps, t_t, loss, vmse))
    info = {"pairs": n, "harvest_grid": "%dx%d" % (a.harvest_n, a.harvest_n), "harvest_seeds": seeds,
            "harvest_steps": a.harvest_steps, "stride": stride, "harvest_s": round(t_h, 2),
            "train_steps": a.train_steps, "batch": a.batch, "train_s": round(t_t, 2),
            "train_mse": round(loss, 5), "heldout_mse": round(vmse, 5),
            "mse_unit": "per-output standardised (1.0 = predicting the mean)",
            "targets": "correction beyond LIN + the stored previous-step correction" if prev else
                       "correction beyond LIN"}
    del train, val
    return mlp, info


def timed_run(name, a, lb, torch, cfg, mom0, mlp, mlp_prev=None):
    prec = lb.FP64 if name.startswith("fp64") else lb.MIXED
    guess = {"eq": lb.GUESS_EQ, "mlp": lb.GUESS_MLP, "lin": lb.GUESS_LIN, "prev": lb.GUESS_PREV,
             "mlpprev": lb.GUESS_MLP_PREV}[name.split("-")[1]]
    stream = torch.cuda.current_stream()
    ctx = lb.Lelbm(cfg, mom0, precision=prec, guess=guess, stream=stream)
    if a.scratch_budget:
        ctx.set_scratch_budget(a.scratch_budget)
    if guess == lb.GUESS_MLP:
        ctx.set_mlp(mlp)
    if guess == lb.GUESS_MLP_PREV:
        ctx.set_mlp(mlp_prev)
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
    mom = ctx.read_moments()
    ctx.close()
    ncell = cfg["nx"] * cfg["ny"]
    prec_name = "fp64" if prec == lb.FP64 else "mixed"
    # per step: the reconstruction and the gather run once per band of the
    # scratch plan
    epr_ms = kt["epr"][0] / a.steps
    gat_ms = kt["gather"][0] / a.steps
    # k_epr handles the cells with unrefined stencils; refined cells go to
    # k_epr_ref (timed apart)
    flops = epr_flops_per_step(st, a.steps)
    # the state the gather writes is FP64 in both modes
    gbytes = (st["arrivals"] / a.steps * GATHER_PAIR_BYTES[prec_name]
              + ncell * (11 * 8 + GATHER_DESC_BYTES))
    r = {
        "mlups": ncell * a.steps / (ms * 1e-3) / 1e6, "ms_per_step": ms / a.steps,
        "epr_ms": epr_ms, "gather_ms": gat_ms, "epr_flops": flops, "gather_bytes": gbytes,
        "epr_tflops": flops / (epr_ms * 1e-3) / 1e12, "gather_gbs": gbytes / (gat_ms * 1e-3) / 1e9,
        "kernels_ms_per_step": {k: round(v[0] / a.steps, 4) for k, v in kt.items() if v[1]},
        "launches_per_step": {k: round(v[1] / a.steps, 2) for k, v in kt.items() if v[1]},
        "lane_occupancy": round(st["point_passes"] / max(st["wave_point_passes"], 1), 4),
        "newton_it": {"mean_f": round(st["it_mean_f"], 3), "max_f": st["it_max_f"],
                      "mean_g": round(st["it_mean_g"], 3), "max_g": st["it_max_g"]},
        "passes_per_cell": round(st["point_passes"] / max(st["q_mean"], 1e-30) / max(st["cells"], 1), 3),
        "refined_share": round(st["point_passes_refined"] / max(st["point_passes"], 1), 5),
        "fallbacks": st["fallbacks"], "stencil_q": {"min": st["q_min"], "mean": round(st["q_mean"], 1),
                                                    "max": st["q_max"]},
        "hbm_bytes": {"persistent": persistent, "scratch": scratch},
    }
    log("%-9s %.2f ms/step  %.1f MLUPS  epr %.3f ms  gather %.3f ms  it %.3f/%.3f  passes %.3f"
        % (name, r["ms_per_step"], r["mlups"], epr_ms, gat_ms, st["it_mean_f"], st["it_mean_g"],
           r["passes_per_cell"]))
    return r, mom


def hotbox_context(lb, li, torch):
    """The paper's only timed workload (uniform advection u = (10, 10),
    4096^2 periodic) on the FP64 path, beside the paper's RTX 4070 times."""
    out = []
    for rt, paper_s in PAPER_HOTBOX_S_PER_STEP.items():
        cfg, prim = li.hotbox(rt, n=4096)
        m = lb.moments_from_primitives(2, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
        c = lb.Lelbm(cfg, m)
        c.step_nostats(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step_nostats(3)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 3
        c.close()
        out.append({"RT": rt, "cells": 4096 * 4096, "s_per_step": round(el, 5),
                    "mlups": round(4096 * 4096 / el / 1e6, 2), "paper_s_per_step": paper_s,
                    "paper_hardware": "RTX 4070 (precision not stated)"})
        log("hot box RT=%.1f: %.4f s/step (paper %.1f s)" % (rt, el, paper_s))
    return out


def channel_run(lb, li, torch, cfg, prim, warmup, steps, label, mlp=None, budget=0):
    """A channel configuration started from rest: after a warm-up that lets the
    bow shocks form, the FP64 path and the FP32 path (with the learned Newton
    guess when a network is given) from the same state, with the relative L1
    error of each field of the FP32 path against the FP64 path on fluid
    cells."""
    m = lb.moments_from_primitives(2, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
    ctx = lb.Lelbm(cfg, m, precision=lb.MIXED if label == "c4" else lb.FP64)
    if budget:
        ctx.set_scratch_budget(budget)
    ctx.step_nostats(warmup)
    torch.cuda.synchronize()
    m0 = ctx.read_moments()
    ctx.close()
    del m
    fluid = cfg["solid"].ravel() == 0
    out, moms = {}, {}
    for name, prec in (("fp64", lb.FP64), ("mixed", lb.MIXED)):
        learned = mlp is not None and prec == lb.MIXED
        c = lb.Lelbm(cfg, m0, precision=prec, guess=lb.GUESS_MLP if learned else lb.GUESS_EQ)
        if learned:
            c.set_mlp(mlp)
        if budget:
            c.set_scratch_budget(budget)
        c.step_nostats(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = c.step(steps)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        persistent, scratch = c.memory()
        moms[name] = c.read_moments()[:, fluid]
        c.close()
        out[name] = {"ms_per_step": round(el * 1e3, 3), "mlups": round(fluid.sum() / el / 1e6, 2),
                     "newton_it": {"mean_f": round(st["it_mean_f"], 3), "max_f": st["it_max_f"],
                                   "mean_g": round(st["it_mean_g"], 3), "max_g": st["it_max_g"]},
                     "stencil_q": {"mean": round(st["q_mean"], 1), "max": st["q_max"]},
                     "reach_max": round(float(st["colat_max"]), 2),
                     "guess": "learned" if learned else "equilibrium", "fallbacks": st["fallbacks"],
                     "hbm_bytes": {"persistent": persistent, "scratch": scratch}}
        log("%s %s: %.2f ms/step %.1f MLUPS q_mean %.1f q_max %d" % (label, name, el * 1e3, out[name]["mlups"],
                                                                      st["q_mean"], st["q_max"]))
    out["l1_mixed_vs_fp64"] = l1_errors(moms["mixed"], moms["fp64"])
    out["config"] = ("channel %dx%d, Mach %.2f inflow (rho 1, RT 1), %d obstacles, started from rest, "
                     "%d warm-up steps, %d timed steps" % (cfg["nx"], cfg["ny"], cfg["mach"],
                                                          len(cfg["obstacles"]), warmup, steps))
    out["fluid_cells"] = int(fluid.sum())
    return out


def channel_context(lb, li, torch, a):
    """The channel configuration: 4096x2048, inflow at the seed's Mach number,
    1-4 seeded elliptical obstacles, slip walls, outflow."""
    cfg, prim = li.channel(a.channel_seed, nx=4096, ny=2048, pad=32)
    out = channel_run(lb, li, torch, cfg, prim, a.channel_warmup, a.channel_steps, "channel",
                      budget=a.scratch_budget)
    out["seed"] = a.channel_seed
    return out


def c4_context(lb, li, torch, a, mlp):
    """The large hypersonic channel: 8192x4096, Mach 10 inflow, eight seeded
    elliptical obstacles (seed 0), pads of 48 cells (the start from rest
    drives a strong shock whose hot gas needs stencils of radius up to ~20).
    The warm-up runs the FP32 path; the bow shocks of the upstream obstacles
    form within it.  The FP32 path then runs with the learned guess (trained
    on four-quadrant runs; cells it does not help fall back to Eq. IID13).
    Reports the HBM footprint: persistent state vs the transient record
    scratch."""
    cfg, prim = li.channel(0, nx=8192, ny=4096, n_obstacles=8, mach=10.0, pad=48)
    out = channel_run(lb, li, torch, cfg, prim, a.c4_warmup, a.c4_steps, "c4", mlp, budget=a.scratch_budget)
    out["seed"] = 0
    return out


def horizon_run(lb, torch, cfg, prim, steps, runs, mlp, label, fluid=None):
    """Two paths from the same initial state for the configuration's own
    number of steps: ms per step of each, and the relative L1 error of each
    field of the second run against the first (the FP64 reference) at the
    end, on fluid cells.  Steps go in chunks of 500 with a progress line."""
    m = lb.moments_from_primitives(2, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
    out, moms = {}, {}
    for name, prec, guess in runs:
        c = lb.Lelbm(cfg, m, precision=prec, guess=guess)
        if guess == lb.GUESS_MLP:
            c.set_mlp(mlp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, qmax, it = 0, 0, 0.0
        while done < steps:
            k = min(500, steps - done)
            st = c.step(k)
            done += k
            qmax = max(qmax, st["q_max"])
            log("%s %s: %d / %d steps, %.1f s" % (label, name, done, steps, time.perf_counter() - t0))
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        persistent, scratch = c.memory()
        mom = c.read_moments()
        moms[name] = mom[:, fluid] if fluid is not None else mom
        c.close()
        out[name] = {"ms_per_step": round(el * 1e3, 3), "q_max": int(qmax), "fallbacks_last_chunk": st["fallbacks"],
                     "hbm_bytes": {"persistent": persistent, "scratch": scratch}}
    first, second = runs[0][0], runs[1][0]
    out["l1_%s_vs_%s" % (second, first)] = l1_errors(moms[second], moms[first])
    out["steps"] = steps
    log("%s: L1 after %d steps %s" % (label, steps, out["l1_%s_vs_%s" % (second, first)]))
    return out


def lockstep_horizon(lb, torch, cfg, prim, steps, runs, mlp, label, fluid, budget, seconds, chunk=250):
    """Two paths from the same initial state advanced in lockstep, `chunk`
    steps at a time, with the relative L1 error of each field of the second
    against the first after every chunk (the error's growth over the
    horizon).  Stops at `steps`, or once the next chunk would pass `seconds`
    of wall time; reports the steps reached."""
    m = lb.moments_from_primitives(2, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
    ctxs = []
    for name, prec, guess in runs:
        c = lb.Lelbm(cfg, m, precision=prec, guess=guess)
        if guess == lb.GUESS_MLP:
            c.set_mlp(mlp)
        if budget:
            c.set_scratch_budget(budget)
        ctxs.append(c)
    del m
    t0 = time.perf_counter()
    done, curve, per = 0, [], {name: 0.0 for name, _, _ in runs}
    qmax = {name: 0 for name, _, _ in runs}
    last = None
    while done < steps:
        k = min(chunk, steps - done)
        if done and time.perf_counter() - t0 + last * k / chunk > seconds:
            break
        tc = time.perf_counter()
        for (name, _, _), c in zip(runs, ctxs):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            st = c.step(k)
            torch.cuda.synchronize()
            per[name] += time.perf_counter() - ts
            qmax[name] = max(qmax[name], st["q_max"])
        done += k
        moms = [c.read_moments()[:, fluid] for c in ctxs]
        e = l1_errors(moms[1], moms[0])
        del moms
        curve.append({"step": done, "l1": {f: float("%.4g" % v) for f, v in e.items()},
                      "q_mean": round(st["q_mean"], 1), "q_max": int(st["q_max"])})
        last = time.perf_counter() - tc
        log("%s: %d / %d steps, %.0f s, L1 rho %.3g u %.3g T %.3g, q_mean %.0f q_max %d"
            % (label, done, steps, time.perf_counter() - t0, e["rho"], e["u"], e["T"], st["q_mean"], st["q_max"]))
    out = {"steps_requested": steps, "steps": done, "l1_curve": curve, "seconds": round(time.perf_counter() - t0, 1)}
    for (name, _, _), c in zip(runs, ctxs):
        persistent, scratch = c.memory()
        out[name] = {"ms_per_step": round(per[name] / max(done, 1) * 1e3, 3), "q_max": qmax[name],
                     "hbm_bytes": {"persistent": persistent, "scratch": scratch}}
        c.close()
    return out


def c0_line(lb, li, torch):
    """The 1D two-state configuration: 2000 cells, seed 0, 1000 steps, on both
    paths, beside the oracle on the host cores for the same 1000 steps."""
    import oracle
    cfg, prim = li.riemann1d(0, n=2000)
    m = lb.moments_from_primitives(1, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
    out, moms = {"workload": "1D two-state, 2000 cells, seed 0, zero-gradient pads of 48, 1000 steps"}, {}
    for name, prec in (("fp64", lb.FP64), ("mixed", lb.MIXED)):
        c = lb.Lelbm(cfg, m, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step_nostats(1000)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        moms[name] = c.read_moments()
        c.close()
        out[name + "_mlups"] = round(2000 * 1000 / el / 1e6, 3)
    r = moms["fp64"][0]
    out["l1_rho_mixed_vs_fp64"] = float(np.abs(moms["mixed"][0] - r).sum() / np.abs(r).sum())
    mo = oracle.moments_from_primitives(1, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
    t0 = time.perf_counter()
    code, ref, _, _ = oracle.step(cfg, mo, 1000)
    el = time.perf_counter() - t0
    out["oracle"] = {"mlups": round(2000 * 1000 / el / 1e6, 4), "cores": oracle.num_threads(), "s": round(el, 2),
                     "status": code}
    out["rel_linf_fp64_vs_oracle"] = float((np.abs(moms["fp64"] - ref).max(axis=1)
                                            / np.maximum(np.abs(ref).max(axis=1), np.abs(ref[0]).max())).max())
    log("C0: fp64 %.2f MLUPS, mixed %.2f MLUPS, oracle %.3f MLUPS (%d threads, %.1f s), GPU vs oracle %.2e"
        % (out["fp64_mlups"], out["mixed_mlups"], out["oracle"]["mlups"], out["oracle"]["cores"], el,
           out["rel_linf_fp64_vs_oracle"]))
    return out


def c1_line(lb, li, torch, mlp):
    """The 1024x1024 four-quadrant configuration, seed 0: the plain FP64 path
    (the configuration's own) and the FP32 path with the learned guess,
    3 warm-up and 20 timed steps each."""
    cfg, prim = li.quadrants(0, n=1024)
    m = lb.moments_from_primitives(2, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
    out = {"workload": "2D four-quadrant 1024x1024 periodic, seed 0, 3 warm-up + 20 timed steps"}
    for name, prec, guess in (("fp64-eq", lb.FP64, lb.GUESS_EQ), ("mixed-mlp", lb.MIXED, lb.GUESS_MLP)):
        c = lb.Lelbm(cfg, m, precision=prec, guess=guess)
        if guess == lb.GUESS_MLP:
            c.set_mlp(mlp)
        c.step_nostats(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = c.step(20)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 20
        c.close()
        out[name] = {"mlups": round(1024 * 1024 / el / 1e6, 2), "ms_per_step": round(el * 1e3, 3),
                     "q_max": st["q_max"], "it_mean_f": round(st["it_mean_f"], 3)}
        log("C1 %s: %.1f MLUPS" % (name, out[name]["mlups"]))
    return out


def d3_line(a, lb, li, torch):
    """The 3D step on an N^3 periodic box with smooth random fields (RT ~ 1,
    mean velocity (0.3, -0.2, 0.1)): FP64 and FP32 records, W warm-up and K
    timed steps each, HIP events on the library's stream, and the oracle on
    a 16^3 box of the same kind on the host cores."""
    import oracle
    n = a.d3
    cfg, prim = li.smooth_periodic3(a.seed, n=n, amp=0.1, RT=1.0)
    m = lb.moments_from_primitives3(cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["uz"], prim["RT"])
    ncell = n ** 3
    out, moms = {}, {}
    for name, prec, guess in (("fp64", lb.FP64, lb.GUESS_EQ), ("mixed", lb.MIXED, lb.GUESS_EQ),
                              ("fp64-lin", lb.FP64, lb.GUESS_LIN), ("mixed-lin", lb.MIXED, lb.GUESS_LIN),
                              ("fp64-prev", lb.FP64, lb.GUESS_PREV), ("mixed-prev", lb.MIXED, lb.GUESS_PREV)):
        stream = torch.cuda.current_stream()
        c = lb.Lelbm(cfg, m, precision=prec, guess=guess, stream=stream)
        if a.scratch_budget:
            c.set_scratch_budget(int(a.scratch_budget))
        c.step_nostats(a.warmup)
        torch.cuda.synchronize()
        c.set_timing(True)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        st = c.step(a.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / a.steps
        kt = c.kernel_times()
        persistent, scratch = c.memory()
        moms[name] = c.read_moments()
        c.close()
        epr_ms = kt["epr"][0] / a.steps
        gat_ms = kt["gather"][0] / a.steps
        flops = epr3_flops_per_step(st, a.steps)
        gbytes = st["arrivals"] / a.steps * GATHER_PAIR_BYTES[name.split("-")[0]] + ncell * (17 * 8 + 28)
        out[name] = {"mlups": round(ncell / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4),
                     "epr_ms": round(epr_ms, 4), "gather_ms": round(gat_ms, 4),
                     "kernels_ms_per_step": {k: round(v[0] / a.steps, 4) for k, v in kt.items() if v[1]},
                     "epr_tflops_executed": round(flops / (epr_ms * 1e-3) / 1e12, 3),
                     "epr_frac_fp64_peak": round(flops / (epr_ms * 1e-3) / 1e12 / VALU_PEAK_TFLOPS, 4),
                     "gather_gbs": round(gbytes / (gat_ms * 1e-3) / 1e9, 1),
                     "newton_it_f": round(st["it_mean_f"], 3), "newton_it_g": round(st["it_mean_g"], 3),
                     "fallbacks": st["fallbacks"], "q_mean": round(st["q_mean"], 1),
                     "q_max": st["q_max"], "hbm_bytes": {"persistent": persistent, "scratch": scratch}}
        log("3D %s: %.2f ms/step, %.1f MLUPS, epr %.3f ms (%.2f TFLOP/s executed), gather %.3f ms"
            % (name, ms, out[name]["mlups"], epr_ms, out[name]["epr_tflops_executed"], gat_ms))
    out["l1_mixed_vs_fp64"] = l1_errors3(moms["mixed"], moms["fp64"])
    out["l1_mixed_lin_vs_fp64"] = l1_errors3(moms["mixed-lin"], moms["fp64"])
    out["l1_fp64_lin_vs_fp64"] = l1_errors3(moms["fp64-lin"], moms["fp64"])
    out["l1_mixed_prev_vs_fp64"] = l1_errors3(moms["mixed-prev"], moms["fp64"])
    out["l1_fp64_prev_vs_fp64"] = l1_errors3(moms["fp64-prev"], moms["fp64"])
    c8, p8 = li.smooth_periodic3(a.seed, n=16, amp=0.1, RT=1.0)
    m8 = oracle.moments_from_primitives3(c8["K"], p8["rho"], p8["ux"], p8["uy"], p8["uz"], p8["RT"])
    t0 = time.perf_counter()
    code, _, _, _ = oracle.step(c8, m8, 4)
    el = time.perf_counter() - t0
    res = {"metric": "MLUPS of the 3D LELBM step (D = 3, 17 stored values)", "value": out["mixed-lin"]["mlups"],
           "unit": "MLUPS", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": out["mixed-lin"]["ms_per_step"], "higher_is_better": True, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "3D periodic box %d^3, smooth random fields (seed %d), RT ~ 1, "
                                  "FP32 records, linearised Newton start" % (n, a.seed),
                      "scratch_budget_bytes": int(a.scratch_budget) if a.scratch_budget else 16 << 30},
           "fp64_mlups": out["fp64"]["mlups"],
           "roofline": {"bound": "alu", "achieved": out["mixed-lin"]["epr_tflops_executed"],
                        "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": out["mixed-lin"]["epr_frac_fp64_peak"],
                        "traffic": stored_traffic("3d").get(("k3_epr", "box%d-mixed-lin" % n)),
                        "kernel": "k3_epr<float> (FP32 records, linearised start)"},
           "cpu_baseline": {"value": round(16 ** 3 * 4 / el / 1e6, 5), "unit": "MLUPS", "cores": oracle.num_threads(),
                            "kind": "oracle", "sample": "16^3 box of the same kind, 4 steps (%.1f s)" % el,
                            "status": code},
           "runs": out}
    return res


def l1_errors3(a, b):
    r = {}
    for name, f in (("rho", lambda m: m[0]), ("u", lambda m: np.sqrt(((m[1:4] / m[0]) ** 2).sum(0))),
                    ("T", lambda m: ((m[4] + m[7] + m[9] + m[13]) / m[0] - ((m[1:4] / m[0]) ** 2).sum(0)) / 5.0)):
        x, y = f(a), f(b)
        r[name] = float(np.abs(x - y).sum() / np.abs(y).sum())
    return r


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
    if a.d3:
        print(json.dumps(d3_line(a, lb, li, torch)), flush=True)
        return
    if a.channel_only:
        print(json.dumps({"channel_context": channel_context(lb, li, torch, a)}), flush=True)
        return
    if a.c4_horizon:
        mlp, _ = harvest_and_train(a, lb, li, torch)
        cfg, prim = li.channel(0, nx=8192, ny=4096, n_obstacles=8, mach=10.0, pad=48)
        kinds = {"fp64-eq": (lb.FP64, lb.GUESS_EQ), "fp64-lin": (lb.FP64, lb.GUESS_LIN),
                 "mixed-mlp": (lb.MIXED, lb.GUESS_MLP), "mixed-eq": (lb.MIXED, lb.GUESS_EQ)}
        pair = tuple((n,) + kinds[n] for n in a.c4_horizon_runs.split(","))
        out = lockstep_horizon(lb, torch, cfg, prim, a.c4_horizon, pair, mlp,
                               "C4", cfg["solid"].ravel() == 0, a.scratch_budget, a.c4_horizon_seconds)
        out["workload"] = ("channel 8192x4096, Mach 10 inflow, 8 obstacles (seed 0), started from rest, "
                           "%d steps" % a.c4_horizon)
        mlp.close()
        print(json.dumps({"c4_horizon": out}), flush=True)
        return
    if a.c4_only:
        mlp, _ = harvest_and_train(a, lb, li, torch)
        out = c4_context(lb, li, torch, a, mlp)
        mlp.close()
        print(json.dumps({"c4_context": out}), flush=True)
        return
    runs = [r for r in a.runs.split(",") if r]
    for r in runs:
        if r not in RUNS:
            raise SystemExit("unknown run %r (choose from %s)" % (r, ", ".join(RUNS)))
    mlp, train_info = (None, None)
    if any(r.endswith("mlp") for r in runs):
        mlp, train_info = harvest_and_train(a, lb, li, torch)
    mlp_prev, train_info_prev = (None, None)
    if any(r.endswith("mlpprev") for r in runs):
        mlp_prev, train_info_prev = harvest_and_train(a, lb, li, torch, prev=True)

    cfg, prim = li.quadrants(a.seed, n=a.n)
    mom0 = lb.moments_from_primitives(2, cfg["K"], prim["rho"], prim["ux"], prim["uy"], prim["RT"])
    res_runs, moms = {}, {}
    for r in runs:
        res_runs[r], moms[r] = timed_run(r, a, lb, torch, cfg, mom0, mlp, mlp_prev)
    ref = "fp64-eq" if "fp64-eq" in moms else None
    for r in runs:
        if ref is not None and r != ref:
            res_runs[r]["l1_vs_fp64"] = l1_errors(moms[r], moms[ref])
    del moms
    head = "mixed-mlp" if "mixed-mlp" in res_runs else runs[0]
    h = res_runs[head]
    traffic = stored_traffic()
    wl = "quadrants%d" % a.n
    ncell = cfg["nx"] * cfg["ny"]
    prec = "fp64" if head.startswith("fp64") else "mixed"
    res = {
        "metric": METRIC,
        "value": round(h["mlups"], 3),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "2D four-quadrant Riemann input %dx%d periodic, seed %d; run %s "
                               "(%s)" % (a.n, a.n, a.seed, head,
                                         "FP32 records, FP64 state, sums and reconstruction, "
                                         "learned Newton guess" if head == "mixed-mlp" else head),
                   "cells": ncell, "warmup_steps": a.warmup},
        "fp64_mlups": round(res_runs["fp64-eq"]["mlups"], 3) if "fp64-eq" in res_runs else None,
        "speedup_vs_fp64": (round(h["mlups"] / res_runs["fp64-eq"]["mlups"], 4)
                            if "fp64-eq" in res_runs else None),
        "l1_vs_fp64": h.get("l1_vs_fp64"),
        "l1_budget": 1e-4,
        "roofline": {"bound": "alu",
                     "kernel": "k_epr (collision, stencil, Newton reconstruction, records; narrow- and "
                               "wide-stencil launches of one step)",
                     "achieved": round(h["epr_tflops"], 3), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(h["epr_tflops"] / VALU_PEAK_TFLOPS, 4),
                     "traffic": traffic.get(("k_epr", wl + "-" + head)),
                     "ms_per_step": round(h["epr_ms"], 4), "flops_per_step": h["epr_flops"],
                     "model": "executed FP64 work of the code (recurrence exponentials), see FLOPS_* in bench.py",
                     "lane_occupancy": h["lane_occupancy"]},
        "gather_roofline": {"bound": "hbm", "kernel": "k_gather", "achieved": round(h["gather_gbs"], 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(h["gather_gbs"] / HBM_PEAK_GBS, 4),
                            "traffic": traffic.get(("k_gather", wl + "-" + head)),
                            "ms_per_step": round(h["gather_ms"], 4), "bytes_per_step": h["gather_bytes"]},
        "runs": {r: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()
                     if k not in ("epr_flops", "gather_bytes")} for r, d in res_runs.items()},
    }
    if train_info is not None:
        res["mlp"] = train_info
    if train_info_prev is not None:
        res["mlp_prev"] = train_info_prev
    if not a.no_context:
        res["c0"] = c0_line(lb, li, torch)
        if mlp is not None:
            res["c1"] = c1_line(lb, li, torch, mlp)
        if a.horizon_steps and mlp is not None:
            res["c2_horizon"] = horizon_run(lb, torch, cfg, prim, a.horizon_steps,
                                            (("fp64-eq", lb.FP64, lb.GUESS_EQ),
                                             ("mixed-mlp", lb.MIXED, lb.GUESS_MLP)), mlp, "C2")
            res["c2_horizon"]["workload"] = ("2D four-quadrant %dx%d periodic, seed %d, %d steps"
                                             % (a.n, a.n, a.seed, a.horizon_steps))
            ccfg, cprim = li.channel(a.channel_seed, nx=4096, ny=2048, pad=32)
            res["c3_horizon"] = horizon_run(lb, torch, ccfg, cprim, a.horizon_steps,
                                            (("fp64-eq", lb.FP64, lb.GUESS_EQ),
                                             ("mixed-eq", lb.MIXED, lb.GUESS_EQ)), None, "C3",
                                            fluid=ccfg["solid"].ravel() == 0)
            res["c3_horizon"]["workload"] = ("channel 4096x2048, seed %d (Mach %.2f, %d obstacles), started "
                                             "from rest, %d steps" % (a.channel_seed, ccfg["mach"],
                                                                      len(ccfg["obstacles"]), a.horizon_steps))
        res["paper_context"] = hotbox_context(lb, li, torch)
        res["channel_context"] = channel_context(lb, li, torch, a)
        if not a.no_c4:
            res["c4_context"] = c4_context(lb, li, torch, a, mlp)
    if mlp is not None:
        mlp.close()
    if mlp_prev is not None:
        mlp_prev.close()
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(cfg, prim, a.cpu_window, a.cpu_steps)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
