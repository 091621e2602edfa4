#!/usr/bin/env python3
"""Throughput of the full-format stray-field apply on one MI355X.

Workload: 128^3 cells on [-1/2, 1/2]^3, smooth vortex magnetization with 5%
seeded noise (seed 0), sinc rule with M = 40 nodes (81-point rule), c0 = 2.15.
One step = one complete apply: potential and all three field components at
every cell (23 mode products per node, all nodes).  Inputs and outputs stay
resident in device memory; the timed region covers only the apply calls.

Prints one JSON line.  ``value`` is cell-field evaluations per second (1e6
cells/s) of the FP64 path; the other precisions are reported beside it with
their relative L2 difference to the FP64 result of the same run.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mcell-field evals/s at 128³, FP64 plain vs mixed+learned R' at rel err 1e-6"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x2": 2500.0, "bf16x3": 2500.0}


def _time_apply(ctx, f, m, phi, h, prec, steps, warmup):
    import torch
    for _ in range(warmup):
        ctx.apply_full(f, m, phi, h, prec=prec)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        ctx.apply_full(f, m, phi, h, prec=prec)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    return ms, prof


def _roofline(prof, prec):
    label, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    per_launch_ms = rec["ms"] / rec["launches"]
    flops = rec["flops"] / rec["launches"]
    achieved = flops / (per_launch_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    return {"bound": "mfma", "kernel": label, "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
            "flops_per_launch": flops, "avg_launch_ms": round(per_launch_ms, 4)}


def _cpu_baseline(m, n, nodes_sample):
    """The oracle's dense-Toeplitz Kronecker apply on the full grid for the
    first `nodes_sample` of the 40 nodes, scaled to all 40."""
    from oracle import apply, sinc
    _t, tau, alpha = sinc.sinc_nodes(40)
    h = (1.0 / n,) * 3
    c0 = time.process_time()
    w0 = time.perf_counter()
    apply.kron_apply_dense(m, h, tau[:nodes_sample], alpha[:nodes_sample])
    wall = time.perf_counter() - w0
    cpu = time.process_time() - c0
    per_apply = wall * 40 / nodes_sample
    return {"value": round(n ** 3 / per_apply / 1e6, 6), "unit": "Mcell-field evals/s",
            "cores": max(1, round(cpu / wall)), "kind": "oracle",
            "sample": f"{nodes_sample} of 40 nodes of the 128^3 vortex apply (FP64 NumPy, dense Toeplitz "
                      f"factors), wall {wall:.1f} s, scaled x{40 / nodes_sample:g}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-nodes", type=int, default=3, help="oracle nodes timed for the CPU baseline (0: skip)")
    ap.add_argument("--precs", default="fp64,fp32,bf16x3,bf16x2")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this library runs on a single GPU; multi-GPU runs are not part of it "
              "(see DESIGN.md for how the path would shard)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1212_3509_amd import api, inputs

    n = 128
    N = n ** 3
    m_host = inputs.vortex_field(n, seed=0)
    ctx = api.Context(0)
    f = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=40, c0=2.15)
    results = {}
    ref = None
    for prec in args.precs.split(","):
        dt = torch.float64 if prec == "fp64" else torch.float32
        m = torch.from_numpy(m_host).to(device="cuda", dtype=dt)
        phi = torch.empty((n, n, n), dtype=dt, device="cuda")
        h = torch.empty((3, n, n, n), dtype=dt, device="cuda")
        ms, prof = _time_apply(ctx, f, m, phi, h, prec, args.steps, args.warmup)
        out = torch.cat([phi.reshape(-1), h.reshape(-1)]).double()
        entry = {"ms_per_step": round(ms, 4), "value": round(N / (ms * 1e-3) / 1e6, 3),
                 "roofline": _roofline(prof, prec),
                 "kernels": {k: {"ms_per_step": round(v["ms"] / args.steps, 4),
                                 "launches_per_step": v["launches"] // args.steps,
                                 "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3)}
                             for k, v in sorted(prof.items())}}
        if ref is None:
            ref = out
        else:
            entry["rel_l2_vs_fp64"] = float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))
        results[prec] = entry
        del m, phi, h
        torch.cuda.empty_cache()

    head = results["fp64"]
    line = {
        "metric": METRIC, "value": head["value"], "unit": "Mcell-field evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "full-format apply, 128^3 vortex + 5% noise (seed 0), sinc rule M=40 "
                               "(81 points), c0=2.15, FP64, potential + field",
                   "cells": N, "nodes": 40},
        "roofline": head["roofline"],
        "precisions": {k: v for k, v in results.items()},
    }
    if args.cpu_nodes > 0:
        line["cpu_baseline"] = _cpu_baseline(m_host, n, args.cpu_nodes)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
