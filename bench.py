#!/usr/bin/env python3
"""Benchmark: 2D Euler MR-HWENO cell-updates/s (FP64) on one MI355X.

Workload: 2D Euler (gamma 1.4), 2048 x 2048 periodic grid on [0, 1]^2, four
seeded constant quadrant states overlaid with an 8-mode smooth Fourier
field, HLLC flux, KXRCF troubled cells (HWENO6-M5-I), CFL 0.6.  One bench
"step" is one SSP-RK3 step of the whole operator (dt reduction, KXRCF
summaries and flags, reconstruction, fluxes, residual and stage combination
for all three stages).  The default times 200 steps, the length of the
configured run, after the state has been reset to t = 0.

Prints one JSON line.  value = cells x RK stages / wall time of the timed
region (inputs resident in HBM).  The timed steps are launched one kernel
at a time with HIP events on the library's stream between kernel classes,
which gives the per-kernel averages of the roofline entry.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, vendor figure
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 vector, vendor figure
# algorithmic HBM traffic of the stage kernel per cell and RK stage (FP64):
# stage 1 reads U^n and writes U^(1) (2 x 96 B); stages 2 and 3 read the
# stage input and U^n and write the output (3 x 96 B): mean 256 B
STAGE_BYTES_PER_CELL = (2 * 96 + 3 * 96 + 3 * 96) / 3.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=2048)
    ap.add_argument("--rows", type=int, default=0, help="2D strip height (0: autotuned/default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration for profiles)")
    return ap.parse_args()


def cpu_baseline(prob, U0):
    """The CPU oracle as it stands, on this host's cores: one evaluation of
    the spatial operator L(U) (one RK stage of work) on the full grid of the
    same workload."""
    import oracle
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.residual(prob, U0)
    dt = time.perf_counter() - t0
    return {"value": prob.ncell / dt, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"one L(U) evaluation (one RK stage) of the full {prob.nx}x{prob.ny} initial state, "
                      f"{dt:.1f} s on {threads} threads"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(the multi-GPU decomposition is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2201_12193_amd import inputs as I
    from paper_2201_12193_amd.mrhweno import Solver

    prob, U0, _ = I.euler_quadrants_2d(seed=args.seed, n=args.n, nq=2)
    dev = torch.device("cuda:0")
    U_init = torch.from_numpy(U0).to(dev)
    Ut = U_init.clone()
    s = Solver([prob], [Ut])
    if args.rows:
        s.set_launch(args.rows, 0)
    # warm-up, then reset to t = 0 so the timed run is the configured run
    s.step(args.warmup)
    s.sync()
    Ut.copy_(U_init)
    torch.cuda.synchronize()
    s.set_time(0, 0.0, 0)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms, nl = s.profile(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t, steps, _ = s.sync()
    if args.calib_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        a.fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        a.sum()                      # read-only pass over 1 GiB
        torch.cuda.synchronize()
        del a, b
    ncell = prob.ncell
    cell_updates = ncell * 3 * args.steps
    value = cell_updates / wall
    stage_ms = ms[3] / max(nl[3], 1)
    achieved_gbs = STAGE_BYTES_PER_CELL * ncell / (stage_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                "kernel": "k2_stage<4,false>", "kernel_avg_ms": stage_ms,
                "kernel_share": ms[3] / max(sum(ms), 1e-9)}
    out = {
        "metric": "2D Euler MR-HWENO cell-updates/s (FP64), plain vs learned-indicator at equal L1",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D Euler quadrants+Fourier {prob.nx}x{prob.ny} periodic, HLLC, KXRCF (M5-I), "
                               f"CFL 0.6, {args.steps} SSP-RK3 steps",
                   "cells": ncell, "rk_stages_per_step": 3, "seed": args.seed,
                   "sim_time": t[0]},
        "kernels_ms": {"reduce_dt": ms[0], "kxrcf_summary": ms[1], "flags": ms[2], "stage": ms[3],
                       "launches": nl},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, U0)
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
