#!/usr/bin/env python3
"""Throughput of the stray-field apply on one MI355X.

Default workload (the headline): 128^3 cells on [-1/2, 1/2]^3, smooth vortex
magnetization with 5% seeded noise (seed 0).  One step = one complete
full-format apply: potential and all three field components at every cell.
Inputs and outputs stay resident in device memory; the timed region covers
only the apply calls.

  * FP64 plain: sinc rule with M = 40 nodes (81-point rule), c0 = 2.15 -> ``value``.
  * mixed + learned: the network is trained on the GPU (outside the timed
    region); its error head picks R' for this grid at the tolerance, the
    shortened rule is fitted and certified (relative Frobenius-norm error of
    the potential and field operators <= tol), and the apply runs with
    bfloat16 three-part split products; its relative L2 difference to the
    FP64 plain result of the same run is reported beside its throughput,
    with the ablation of the network (R', fits and time of each predict
    mode) and the plain rule's node count at the same certified tolerance.
  * FP32, BF16x3 and BF16x2 with the full rule, for reference.
  * Sub-records of the same line: the 3D-FFT route, a graded non-uniform
    grid, the structured applies at n = 4096 (CP rank 10, Tucker (8,8,8), TT
    (1,8,8,1); M = 40 and the certified theorem-step rule with 64 nodes) and
    the batch of 256 uneven states, each with its roofline, and the CPU
    oracle baseline (1 core and all cores, median of 3).

``--workload cp4096`` / ``batch`` print only those sub-records.
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
KERNEL_SOURCES = ("paper_1212_3509_amd/csrc/modeprod.hip", "paper_1212_3509_amd/csrc/modeprod_bf16.hip",
                  "paper_1212_3509_amd/csrc/internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_full_apply_128_vortex.json")
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x2": 2500.0, "bf16x3": 2500.0}
HBM_GBS = 8000.0
# vector-ALU peaks (TFLOP/s): FP64, and FP32 as published (packed FP32 counted)
FP64_VEC_TFLOPS = 78.6
FP32_VEC_TFLOPS = 157.3


_T0 = time.perf_counter()


def _progress(msg):
    """One line on stderr per finished part of the run (long runs show progress)."""
    print(f"bench: {msg} ({time.perf_counter() - _T0:.1f} s)", file=sys.stderr, flush=True)


def _timed(ctx, fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    return ms, prof


def _kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _traffic(label):
    """HBM bytes per launch of `label` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size), or
    None when it is missing or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != _kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(label)
    return None if k is None else k["hbm_bytes_per_launch"]


def write_traffic(fetch_csv, write_csv, calib_mib):
    """Rewrite the counter summary from two rocprofv3 --pmc runs (FETCH_SIZE,
    then WRITE_SIZE, KiB per dispatch) of the FP64 headline with a plain copy
    of `calib_mib` MiB first.  The stage labels keep their kernel names from
    the existing summary; each stage's counters are the median over its
    dispatches, scaled by what the counters read for the copy."""
    import csv
    import statistics

    def per_kernel(path, counter):
        vals = {}
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return vals

    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    nbytes = calib_mib << 20
    # the copy: of the elementwise kernels that write its byte count (the
    # fill of its source does too), the one that also reads
    copy = [k for k, v in write.items() if "elementwise" in k and abs(max(v) * 1024 - nbytes) < 0.01 * nbytes]
    if not copy:
        raise SystemExit("write_traffic: calibration copy not found")
    copy = max(copy, key=lambda k: max(fetch.get(k, [0.0])))
    fk, wk = max(fetch[copy]), max(write[copy])
    cal = {"bytes": nbytes, "fetch_kib": fk, "write_kib": wk, "fetch_scale": nbytes / (fk * 1024),
           "write_scale": nbytes / (wk * 1024)}
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    def lookup(vals, kernel):   # full demangled names: "...::k_left<double, 8, 2, 2, true>(args)"
        hits = [v for name, v in vals.items() if "::" + kernel + "(" in name]
        if len(hits) != 1:
            raise SystemExit(f"write_traffic: {len(hits)} dispatches groups match {kernel}")
        return statistics.median(hits[0])

    for label, k in rec["kernels"].items():
        f = lookup(fetch, k["kernel"])
        w = lookup(write, k["kernel"])
        k.update({"fetch_kib": f, "write_kib": w,
                  "hbm_bytes_per_launch": 1024 * (f * cal["fetch_scale"] + w * cal["write_scale"])})
    rec["copy_calibration"] = cal
    rec["kernel_source_sha256"] = _kernel_source_hash()
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


def _roofline(prof, prec):
    label, rec = max(prof.items(), key=lambda kv: kv[1]["ms"])
    per_launch_ms = rec["ms"] / rec["launches"]
    flops = rec["flops"] / rec["launches"]
    achieved = flops / (per_launch_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[prec]
    return {"bound": "mfma", "kernel": label, "achieved": round(achieved, 3), "peak": peak,
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": _traffic(label),
            "traffic_unit": "bytes per launch", "flops_per_launch": flops,
            "algorithmic_bytes_per_launch": rec["bytes"] / rec["launches"], "avg_launch_ms": round(per_launch_ms, 4)}


def _copy_calibration(mib):
    """A plain elementwise copy of `mib` MiB (read once, written once): the
    reference dispatch for scaling the HBM byte counters."""
    import torch
    x = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    del x, y


def _vendor_gemm():
    """Context for the matrix-core figures: torch.matmul (the vendor GEMM
    library) on square contiguous matrices, FP64 / FP32 / BF16, TFLOP/s of
    the best of three timed calls."""
    import torch
    out = {}
    for name, dt, size in (("fp64", torch.float64, 8192), ("fp32", torch.float32, 8192), ("bf16", torch.bfloat16, 16384)):
        a = torch.rand((size, size), dtype=dt, device="cuda")
        b = torch.rand((size, size), dtype=dt, device="cuda")
        c = torch.matmul(a, b)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            torch.matmul(a, b, out=c)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[name] = {"n": size, "tflops": round(2.0 * size ** 3 / (best * 1e-3) / 1e12, 1)}
        del a, b, c
        torch.cuda.empty_cache()
    return out


def _kernels(prof, steps):
    return {k: {"ms_per_step": round(v["ms"] / steps, 4), "launches_per_step": v["launches"] // steps,
                "tflops": round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 3)} for k, v in sorted(prof.items())}


def _median_wall(fn, runs):
    """Median wall time of `runs` calls and the CPU threads busy during them."""
    walls, cpus = [], []
    for _ in range(runs):
        c0, w0 = time.process_time(), time.perf_counter()
        fn()
        walls.append(time.perf_counter() - w0)
        cpus.append(time.process_time() - c0)
    i = sorted(range(runs), key=lambda j: walls[j])[runs // 2]
    return walls[i], cpus[i]


def _cpu_baseline(m, n, runs):
    """The oracle timed on this host's cores: its dense-Toeplitz Kronecker
    apply (FP64 NumPy) of the 128^3 vortex on a node sample, scaled to the 40
    nodes of the rule (the apply is a sum over nodes).  One core: one node
    per run.  All cores: the oracle run unchanged on one node per core in a
    thread pool (its einsum loops release the interpreter lock).  Median of
    `runs` runs each.  Beside it, each at one core and all cores: the exact
    collocation (closed-form cell kernels + FFT convolution) at 32^3 and, on
    samples, at 128^3; the Kronecker method at 32^3; the batch of 256 uneven
    states on a sample of states; and the structured reference (dense
    Toeplitz products of the factor columns) at n = 4096 for CP rank 10,
    Tucker (8,8,8) and TT (1,8,8,1) inputs, on one component and node per
    axis, scaled to the whole apply."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    from scipy import fft as sfft
    from threadpoolctl import threadpool_limits

    from oracle import apply, exact, sinc, structured
    from paper_1212_3509_amd import inputs
    _t, tau, alpha = sinc.sinc_nodes(40)
    h = (1.0 / n,) * 3
    cores = len(os.sched_getaffinity(0))
    wall1, cpu1 = _median_wall(lambda: apply.kron_apply_dense(m, h, tau[:1], alpha[:1]), runs)

    def all_cores():
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda k: apply.kron_apply_dense(m, h, tau[k % 40:k % 40 + 1], alpha[k % 40:k % 40 + 1]),
                        range(cores)))
    wallc, cpuc = _median_wall(all_cores, runs)
    per_apply_1 = wall1 * 40
    per_apply_c = wallc * 40 / cores
    out = {"value": round(n ** 3 / per_apply_c / 1e6, 6), "unit": "Mcell-field evals/s",
           "cores": max(1, round(cpuc / wallc)), "kind": "oracle",
           "sample": f"oracle dense-Toeplitz Kronecker apply (FP64 NumPy) of the 128^3 vortex, one node per "
                     f"thread on {cores} threads, median of {runs}: {wallc:.2f} s for {cores} of the 40 nodes, "
                     f"scaled to 40",
           "one_core": {"value": round(n ** 3 / per_apply_1 / 1e6, 6), "unit": "Mcell-field evals/s",
                        "cores": max(1, round(cpu1 / wall1)),
                        "sample": f"one node, median of {runs}: {wall1:.2f} s, scaled x40"}}
    out["host"] = _host_info()
    m32 = inputs.random_unit_field(32, seed=0)
    h32 = (1.0 / 32,) * 3
    wall, cpu = _median_wall(lambda: apply.collocated_apply_fft(m32, h32), runs)

    def exact32_all():
        with sfft.set_workers(cores):
            apply.collocated_apply_fft(m32, h32)
    wallc32, cpuc32 = _median_wall(exact32_all, runs)
    out["exact_fft_32"] = {"value": round(32 ** 3 / wall / 1e6, 6), "unit": "Mcell-field evals/s",
                           "seconds": round(wall, 3), "cores": max(1, round(cpu / wall)),
                           "all_cores": {"value": round(32 ** 3 / wallc32 / 1e6, 6), "seconds": round(wallc32, 3),
                                         "cores": max(1, round(cpuc32 / wallc32)),
                                         "sample": f"the same with scipy.fft's workers = {cores}"}}
    # the Kronecker method at 32^3, all 40 nodes: one core, and one node per
    # thread in a pool of all cores
    with threadpool_limits(1):
        wk32, ck32 = _median_wall(lambda: apply.kron_apply_dense(m32, h32, tau, alpha), runs)

    def kron32_all():
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda k: apply.kron_apply_dense(m32, h32, tau[k:k + 1], alpha[k:k + 1]), range(40)))
    wkc32, ckc32 = _median_wall(kron32_all, runs)
    out["kron_32"] = {"value": round(32 ** 3 / wkc32 / 1e6, 6), "unit": "Mcell-field evals/s",
                      "seconds": round(wkc32, 3), "cores": max(1, round(ckc32 / wkc32)),
                      "one_core": {"value": round(32 ** 3 / wk32 / 1e6, 6), "seconds": round(wk32, 3),
                                   "cores": max(1, round(ck32 / wk32))},
                      "sample": f"oracle dense-Toeplitz Kronecker apply (FP64 NumPy) of a random unit field at "
                                f"32^3, all 40 nodes (one core: BLAS limited to one thread; all cores: one node "
                                f"per thread on {cores} threads), median of {runs}"}
    # exact collocation at 128^3: closed-form cell kernels on all 255^3
    # offsets, then 12 FFT convolutions of 255^3 kernels with 128^3 fields
    # (3 for phi, 9 for h).  Timed on samples scaled to the whole: the
    # kernels of 7 of the 255 z-offset planes (the 128 x 128 x 4 grid; the
    # cost per offset does not depend on it) and one of the convolutions.
    # All cores: one kernel sample per thread (its planes stand for 7 more),
    # the convolution with scipy.fft's workers.
    h128 = (1.0 / n,) * 3
    ker = np.random.default_rng(3).standard_normal((2 * n - 1,) * 3)
    wk1, ck1 = _median_wall(lambda: exact.offset_kernels((n, n, 4), h128), runs)
    wv1, cv1 = _median_wall(lambda: apply._linear_conv_same(ker, m[0]), runs)

    def kern_all():
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda _i: exact.offset_kernels((n, n, 4), h128), range(cores)))

    def conv_all():
        with sfft.set_workers(cores):
            apply._linear_conv_same(ker, m[0])
    wkc, ckc = _median_wall(kern_all, runs)
    wvc, cvc = _median_wall(conv_all, runs)
    del ker
    planes = 2 * n - 1
    t1 = wk1 * planes / 7 + wv1 * 12
    tc = wkc * planes / (7 * cores) + wvc * 12
    out["exact_fft_128"] = {
        "value": round(n ** 3 / tc / 1e6, 6), "unit": "Mcell-field evals/s", "seconds_per_apply": round(tc, 2),
        "cores": max(1, round((ckc + cvc) / (wkc + wvc))),
        "one_core": {"value": round(n ** 3 / t1 / 1e6, 6), "seconds_per_apply": round(t1, 2),
                     "cores": max(1, round((ck1 + cv1) / (wk1 + wv1)))},
        "sample": f"oracle exact collocation (closed-form kernels + FFT convolution, FP64): kernels of 7 of "
                  f"{planes} offset planes ({wk1:.2f} s on one core, {wkc:.2f} s for {cores} threads' samples) "
                  f"scaled x{planes / 7:.1f}, one of 12 convolutions ({wv1:.2f} s on one core, {wvc:.2f} s "
                  f"with {cores} workers) scaled x12; median of {runs}"}
    # structured reference at n = 4096: the oracle's columns of one axis,
    # component and node (two dense Toeplitz products, FP64 BLAS) for the
    # column counts of each format, scaled to 3 components x 40 nodes and
    # summed over the axes (CP rank 10: 10 columns per axis; Tucker
    # (8,8,8): 8; TT (1,8,8,1): 8, 64, 8); one core (BLAS limited to one
    # thread) and all cores
    N4 = 4096
    F = sinc.scaled_factors(N4, 1.0 / N4, tau[:1], alpha[:1])
    rng4 = np.random.default_rng(1)
    widths = {"cp_r10": (10, 10, 10), "tucker_888": (8, 8, 8), "tt_188_1": (8, 64, 8)}
    cols = {w: rng4.uniform(-1, 1, (N4, w)) for w in (8, 10, 64)}
    for name, ws in widths.items():
        rec = {}
        for label, limit in (("one_core", 1), ("all_cores", None)):
            per_apply = 0.0
            cpu_tot = wall_tot = 0.0
            for w in ws:
                with threadpool_limits(limit):
                    wall, cpu = _median_wall(lambda w=w: structured._columns(F, 0, 0, cols[w], 1), runs)
                per_apply += wall * 3 * 40
                wall_tot += wall
                cpu_tot += cpu
            rec[label] = {"value": round(N4 ** 3 / per_apply / 1e12, 6), "unit": "implicit Tcell/s",
                          "seconds_per_apply": round(per_apply, 3), "cores": max(1, round(cpu_tot / wall_tot))}
        out[f"structured_4096_{name}"] = dict(rec["all_cores"], one_core=rec["one_core"],
                                              sample=f"the oracle's columns of one component and node per axis "
                                                     f"({'/'.join(str(w) for w in ws)} columns, two dense 4096 x "
                                                     f"4096 Toeplitz products each, FP64 BLAS), median of {runs}, "
                                                     f"scaled x120 (3 components, 40 nodes) and summed over the axes")
    # the batch of 256 uneven states: the Kronecker method on a sample of
    # states (one node each), scaled by the ratio of the mode-product work
    # sum_s N_s (nx + ny + nz) of the whole batch to the sample's, and by 40
    # nodes; one core, and the sample's (state, node) pairs on a pool of all
    # cores
    states = inputs.batch_grids(256, seed=2, with_fields=False)
    work = lambda st: float(np.prod(st.n)) * sum(st.n)  # noqa: E731
    pick = [0, 3, 15, 23]   # two cubes, films with 8 and 16 cells across
    sample = [(states[i].n, states[i].h, inputs.random_unit_field(states[i].n, seed=states[i].seed)) for i in pick]
    scale = sum(work(st) for st in states) / sum(work(states[i]) for i in pick) * 40
    cells = sum(int(np.prod(st.n)) for st in states)

    def batch_one():
        for nn, hh, mm in sample:
            apply.kron_apply_dense(mm, hh, tau[:1], alpha[:1])
    with threadpool_limits(1):
        wb1, cb1 = _median_wall(batch_one, runs)

    def batch_all():
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda t: apply.kron_apply_dense(sample[t[0]][2], sample[t[0]][1], tau[t[1]:t[1] + 1],
                                                         alpha[t[1]:t[1] + 1]),
                        [(i, k) for i in range(len(sample)) for k in range(cores // len(sample) or 1)]))
    wbc, cbc = _median_wall(batch_all, runs)
    per_node_all = wbc / (cores // len(sample) or 1)
    out["batch_256"] = {"value": round(cells / (per_node_all * scale) / 1e6, 6), "unit": "Mcell-field evals/s",
                        "seconds_per_batch": round(per_node_all * scale, 1), "cores": max(1, round(cbc / wbc)),
                        "one_core": {"value": round(cells / (wb1 * scale) / 1e6, 6),
                                     "seconds_per_batch": round(wb1 * scale, 1), "cores": max(1, round(cb1 / wb1))},
                        "sample": f"oracle dense-Toeplitz Kronecker apply (FP64 NumPy) of states {pick} (grids "
                                  f"{[states[i].n for i in pick]}), one node each, median of {runs}, scaled "
                                  f"x{scale:.0f} by the mode-product work of the 256 states and the 40 nodes; all "
                                  f"cores: {cores // len(sample) or 1} nodes per sampled state on {cores} threads"}
    return out


def _host_info():
    """Host cores and BLAS threading of the process that timed the oracle."""
    import os
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as fh:
            info["cpu_model"] = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        info["cpu_model"] = None
    try:
        import threadpoolctl
        info["blas"] = [{"api": d.get("internal_api"), "threads": d.get("num_threads")}
                        for d in threadpoolctl.threadpool_info()]
    except ImportError:
        info["blas"] = None
    return info


def _rel(a, b):
    import torch
    return float(torch.linalg.norm((a - b).reshape(-1)) / torch.linalg.norm(b.reshape(-1)))


def _judge(ctx, n, t, alpha):
    """Certified operator error of the rule (t, alpha) on the n^3 unit cube:
    the larger of the potential's and the field's relative Frobenius-norm
    errors against the 96-node theorem-step rule."""
    return max(ctx.quad_certify((n, n, n), (1.0 / n,) * 3, t, alpha))


def _learned_eval(ctx, params, args):
    """The trained network on grids beyond its training range: 256^3 full
    format (vortex) and 1024^3 CP rank 10; each uses the predicted rule, or
    the fallback rule when no shortened rule is certified within the
    tolerance.  Every rule's certificate (larger of the potential's and the
    field's operator errors) is reported beside the measured errors."""
    import numpy as np
    import torch

    from paper_1212_3509_amd import inputs, learned
    out = {}
    # 256^3 full format
    n = 256
    N = n ** 3
    rule = learned.predict(ctx, params, (n, n, n), args.rule_tol, fit_iters=args.predict_iters)
    fr = ctx.assemble((n, n, n), (1.0 / n,) * 3, t=rule["t"], alpha=rule["alpha"])
    fp = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=40, c0=2.15)
    pt, _ptau, pa = fp.nodes()
    m_host = inputs.vortex_field(n, seed=0)
    rec = {"nodes": rule["R"], "fell_back": rule["fell_back"], "fits": rule["fits"], "rule_tol": args.rule_tol,
           "rule_certified_err": rule["judged"], "plain_m40_certified_err": _judge(ctx, n, pt, pa),
           "predict_seconds": round(rule["seconds"], 3)}
    # accurate reference: the theorem-step rule with 64 nodes (the fallback rule)
    fa = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=64, step_rule=1)
    at, _atau, aa = fa.nodes()
    rec["reference_theorem_m64_certified_err"] = _judge(ctx, n, at, aa)
    runs = {}
    ref = None
    for name, f, prec in (("reference_theorem_m64_fp64", fa, "fp64"), ("rule_fp64", fr, "fp64"),
                          ("rule_" + args.mixed_prec, fr, args.mixed_prec), ("plain_m40_fp64", fp, "fp64")):
        dt = torch.float64 if prec == "fp64" else torch.float32
        m = torch.from_numpy(m_host).to(device="cuda", dtype=dt)
        phi = torch.empty((n, n, n), dtype=dt, device="cuda")
        h = torch.empty((3, n, n, n), dtype=dt, device="cuda")
        ms, _prof = _timed(ctx, lambda: ctx.apply_full(f, m, phi, h, prec=prec), 2, 1)
        r = {"ms_per_step": round(ms, 3), "value": round(N / (ms * 1e-3) / 1e6, 3)}
        if ref is None:
            ref = (phi.double().clone(), h.double().clone())
        else:
            r["rel_l2_vs_reference"] = {"phi": _rel(phi.double(), ref[0]), "h": _rel(h.double(), ref[1])}
        runs[name] = r
        del m, phi, h
        torch.cuda.empty_cache()
    rec["applies"] = runs
    out["full_256"] = rec
    del ref, fr, fp, fa
    torch.cuda.empty_cache()
    # 1024^3 CP rank 10 (structured)
    n = 1024
    rule = learned.predict(ctx, params, (n, n, n), args.rule_tol, fit_iters=args.predict_iters)
    fr = ctx.assemble((n, n, n), (1.0 / n,) * 3, t=rule["t"], alpha=rule["alpha"])
    fp = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=40, c0=2.15)
    pt, _ptau, pa = fp.nodes()
    cp = inputs.cp_input(n, rank=10, seed=1, dtype=np.float32)
    U = [torch.from_numpy(np.ascontiguousarray(np.stack([cp.U[q][d].T for q in range(3)]))).cuda()
         for d in range(3)]
    rec = {"nodes": rule["R"], "fell_back": rule["fell_back"], "fits": rule["fits"], "rule_tol": args.rule_tol,
           "rule_certified_err": rule["judged"], "plain_m40_certified_err": _judge(ctx, n, pt, pa),
           "predict_seconds": round(rule["seconds"], 3)}
    for name, f in (("rule", fr), ("plain_m40", fp)):
        ctx.prepare_structured(f)
        ms, _prof = _timed(ctx, lambda: ctx.apply_cp(f, U), 3, 1)
        rec[name] = {"ms_per_apply": round(ms, 4), "implicit_cells_per_s": n ** 3 / (ms * 1e-3)}
    out["cp_1024_r10"] = rec
    return out


def headline(args):
    import numpy as np
    import torch

    from paper_1212_3509_amd import api, inputs, learned

    n = 128
    N = n ** 3
    m_host = inputs.vortex_field(n, seed=0)
    if args.calib_copy_mib > 0:
        _copy_calibration(args.calib_copy_mib)
    ctx = api.Context(0)
    f = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=40, c0=2.15)
    results = {}
    ref = None
    # FP64 first: it is the headline and the reference of the other precisions
    for prec in ["fp64"] + [p for p in args.precs.split(",") if p and p != "fp64"]:
        dt = torch.float64 if prec == "fp64" else torch.float32
        m = torch.from_numpy(m_host).to(device="cuda", dtype=dt)
        phi = torch.empty((n, n, n), dtype=dt, device="cuda")
        h = torch.empty((3, n, n, n), dtype=dt, device="cuda")
        ms, prof = _timed(ctx, lambda: ctx.apply_full(f, m, phi, h, prec=prec), args.steps, args.warmup)
        entry = {"ms_per_step": round(ms, 4), "value": round(N / (ms * 1e-3) / 1e6, 3),
                 "roofline": _roofline(prof, prec), "kernels": _kernels(prof, args.steps)}
        if ref is None:
            ref = (phi.double().clone(), h.double().clone())
        else:
            entry["rel_l2_vs_fp64"] = {"phi": _rel(phi.double(), ref[0]), "h": _rel(h.double(), ref[1])}
        results[prec] = entry
        del m, phi, h
        torch.cuda.empty_cache()
        _progress(f"{prec} apply timed")

    # the same operator by 3D FFT convolution (Sec. 4.2's route for full tensors)
    fft3d = None
    if args.fft3d:
        m = torch.from_numpy(m_host).to(device="cuda", dtype=torch.float64)
        phi = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        h = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
        ms, prof = _timed(ctx, lambda: ctx.apply_fft(f, m, phi, h), args.steps, args.warmup)
        rec = prof["fft3d/fp64"]
        fft3d = {"value": round(N / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4), "dtype": "f64",
                 "rel_l2_vs_mode_products": {"phi": _rel(phi, ref[0]), "h": _rel(h, ref[1])},
                 "algorithmic_GBps": round(rec["bytes"] / rec["launches"] / (rec["ms"] / rec["launches"] * 1e-3) / 1e9, 1),
                 "hbm_frac": round(rec["bytes"] / (rec["ms"] * 1e-3) / 1e9 / HBM_GBS, 4)}
        del m, phi, h
        torch.cuda.empty_cache()
        _progress("3D-FFT route timed")

    # the same operator on a non-uniform grid (graded cells, dense factors)
    nonuni = None
    if args.nonuniform:
        edges = []
        for r in (1.01, 0.99, 1.005):
            w = r ** np.arange(n)
            e = np.concatenate([[0.0], np.cumsum(w)])
            edges.append(e / e[-1] - 0.5)
        fn = ctx.assemble_grid(edges, M=40, c0=2.15)
        m = torch.from_numpy(m_host).to(device="cuda", dtype=torch.float64)
        phi = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        h = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda")
        ms, prof = _timed(ctx, lambda: ctx.apply_full(fn, m, phi, h, prec="fp64"), max(2, args.steps // 2), 1)
        nonuni = {"value": round(N / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4), "dtype": "f64",
                  "grid": "128^3 graded cells (width ratios 1.01, 0.99, 1.005 per cell), M=40",
                  "roofline": _roofline(prof, "fp64"), "kernels": _kernels(prof, max(2, args.steps // 2))}
        # the same in FP32 (dense tables rounded once from FP64) and BF16x3
        # (tables split into three bfloat16 parts), against the FP64 result
        m32 = m.float()
        phi32 = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        h32 = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
        rel = lambda a, b: float(torch.linalg.norm((a.double() - b).reshape(-1)) / torch.linalg.norm(b.reshape(-1)))  # noqa: E731
        for prec in ("fp32", "bf16x3"):
            ms32, prof32 = _timed(ctx, lambda: ctx.apply_full(fn, m32, phi32, h32, prec=prec),
                                  max(2, args.steps // 2), 1)
            nonuni[prec] = {"value": round(N / (ms32 * 1e-3) / 1e6, 3), "ms_per_step": round(ms32, 4),
                            "dtype": "f32" if prec == "fp32" else prec,
                            "rel_l2_vs_fp64": {"phi": rel(phi32, phi), "h": rel(h32, h)},
                            "roofline": _roofline(prof32, prec), "kernels": _kernels(prof32, max(2, args.steps // 2))}
        del m, phi, h, fn, m32, phi32, h32
        torch.cuda.empty_cache()
        _progress("non-uniform grid timed")

    mixed = None
    if args.learned_steps > 0:
        t0 = time.perf_counter()
        cases = learned.prepare_cases(args.cases, seed=3)
        learned.fit_targets(ctx, cases, iters=args.fit_iters)
        torch.cuda.synchronize()
        fit_s = time.perf_counter() - t0
        _progress("training targets fitted")
        params, loss = learned.train(ctx, cases, steps=args.learned_steps, batch=512)
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0 - fit_s
        _progress("network trained")
        # what the network contributes: the three predict modes at this grid
        ablation = {}
        for mode in ("network", "network_proposal", "search"):
            r = learned.predict(ctx, params, (n, n, n), args.rule_tol, fit_iters=args.predict_iters, mode=mode)
            ablation[mode] = {k: r[k] for k in ("R", "fell_back", "fits", "err_phi", "err_h", "seconds",
                                                "accuracy_met")}
            if mode == "network":
                rule = r
            _progress(f"predict ({mode}) done")
        # the plain sinc rule's node count for the same certified tolerance
        # (nodes from the library's own assembly)
        plain_nodes = None
        for M in range(16, 65):
            fM = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=M, c0=2.15)
            t_, _tau, a_ = fM.nodes()
            fM.free()
            if _judge(ctx, n, t_, a_) <= args.rule_tol:
                plain_nodes = M
                break
        fl = ctx.assemble((n, n, n), (1.0 / n,) * 3, t=rule["t"], alpha=rule["alpha"])
        m = torch.from_numpy(m_host).to(device="cuda", dtype=torch.float32)
        phi = torch.empty((n, n, n), dtype=torch.float32, device="cuda")
        h = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
        prec = args.mixed_prec
        ms, prof = _timed(ctx, lambda: ctx.apply_full(fl, m, phi, h, prec=prec), args.steps, args.warmup)
        err = {"phi": _rel(phi.double(), ref[0]), "h": _rel(h.double(), ref[1])}
        mixed = {"value": round(N / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms, 4), "dtype": prec,
                 "nodes": rule["R"], "fell_back": rule["fell_back"], "rule_tol": args.rule_tol,
                 "certified": {"phi": rule["err_phi"], "h": rule["err_h"]},
                 "predicted_log10_err": rule["predicted"],
                 "rel_l2_vs_fp64_plain": err, "meets_1e-6": max(err.values()) <= 1e-6,
                 "speedup_vs_fp64_plain": round(results["fp64"]["ms_per_step"] / ms, 3),
                 "plain_sinc_nodes_for_rule_tol": plain_nodes,
                 "node_ratio_vs_plain_sinc": None if plain_nodes is None else round(rule["R"] / plain_nodes, 3),
                 "ablation": ablation,
                 "roofline": _roofline(prof, prec), "kernels": _kernels(prof, args.steps),
                 "training": {"cases": args.cases, "fit_iters": args.fit_iters, "fit_seconds": round(fit_s, 2),
                              "median_fitted_log10_err": float(np.median(np.log10(cases["fit_err"].cpu().numpy()))),
                              "steps": args.learned_steps, "train_seconds": round(train_s, 2),
                              "loss_first": float(loss[:10].mean()), "loss_last": float(loss[-10:].mean()),
                              "predict_fit_iters": args.predict_iters}}
        del m, phi, h, fl
        torch.cuda.empty_cache()

    learned_eval = None
    if args.learned_steps > 0 and args.learned_eval:
        _progress("mixed + learned apply timed")
        learned_eval = _learned_eval(ctx, params, args)

    del f
    torch.cuda.empty_cache()
    _progress("learned rule done")
    structured_rec = structured_record(ctx, args) if args.structured else None
    _progress("structured applies timed")
    tucker_rec = tucker_record(ctx, args) if args.tucker else None
    _progress("Tucker route timed")
    del ctx
    torch.cuda.empty_cache()
    batch_rec = batch_record(args) if args.batch else None
    _progress("batch timed")

    head = results["fp64"]
    # the apply's compulsory traffic (m in, phi and h out) beside what the
    # counters read for its stage launches
    algo = 7.0 * N * 8
    counted = [_traffic(k) for k in head["kernels"]]
    head["roofline"]["apply_bytes"] = {
        "algorithmic_7N": algo,
        "counters": None if any(c is None for c in counted) else sum(counted),
        "ratio": None if any(c is None for c in counted) else round(sum(counted) / algo, 2)}
    line = {
        "metric": METRIC, "value": head["value"], "unit": "Mcell-field evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "full-format apply, 128^3 vortex + 5% noise (seed 0), sinc rule M=40 "
                               "(81 points), c0=2.15, FP64, potential + field",
                   "cells": N, "nodes": 40},
        "roofline": head["roofline"],
        "mixed_learned": mixed,
        "learned_eval": learned_eval,
        "fft3d_route": fft3d,
        "nonuniform_grid": nonuni,
        "structured_4096": structured_rec,
        "tucker_route": tucker_rec,
        "batch_256": batch_rec,
        "precisions": results,
    }
    if args.vendor_gemm:
        line["vendor_gemm"] = _vendor_gemm()
    _progress("vendor GEMM context done")
    if args.cpu_runs > 0:
        line["cpu_baseline"] = _cpu_baseline(m_host, n, args.cpu_runs)
        _progress("CPU baseline done")
    print(json.dumps(line), flush=True)


def structured_record(ctx, args):
    """Structured applies at n = 4096 per axis (CP rank 10, Tucker (8,8,8),
    TT (1,8,8,1)), with the rule M = 40 (c0 = 2.15) and the theorem-step rule
    with 64 nodes, each rule's certificate, the HOOI recompression of the CP
    potential, and the roofline of the transform launches (HBM bound: the
    algorithmic bytes are the input and output columns plus the kernel
    spectra, per apply)."""
    import numpy as np
    import torch

    from paper_1212_3509_amd import inputs

    n, M = 4096, 40
    f = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=M, c0=2.15)
    ctx.prepare_structured(f)
    out = {}
    cp = inputs.cp_input(n, rank=10, seed=1, dtype=np.float32)
    U = [torch.from_numpy(np.ascontiguousarray(np.stack([cp.U[q][d].T for q in range(3)]))).cuda() for d in range(3)]
    tk = inputs.tucker_input(n, ranks=(8, 8, 8), seed=1, dtype=np.float32)
    V = [torch.from_numpy(np.ascontiguousarray(np.stack([tk.U[q][d].T for q in range(3)]))).cuda() for d in range(3)]
    tt = inputs.tt_input(n, ranks=(8, 8), seed=1, dtype=np.float32)
    G1 = torch.from_numpy(np.ascontiguousarray(np.stack([tt.G1[q].T for q in range(3)]))).cuda()
    G2 = torch.from_numpy(np.ascontiguousarray(np.stack([tt.G2[q].transpose(0, 2, 1) for q in range(3)]))).cuda()
    G3 = torch.from_numpy(np.ascontiguousarray(np.stack([tt.G3[q] for q in range(3)]))).cuda()
    fa = ctx.assemble((n, n, n), (1.0 / n,) * 3, M=64, step_rule=1)
    ctx.prepare_structured(fa)
    t40, _tau, a40 = f.nodes()
    t64, _tau, a64 = fa.nodes()
    certified = {"m40_c0_2.15": ctx.quad_certify((n, n, n), (1.0 / n,) * 3, t40, a40),
                 "theorem_m64": ctx.quad_certify((n, n, n), (1.0 / n,) * 3, t64, a64)}
    cases = {}
    for prec in ("fp64", "fp32"):
        for rname, ff in (("", f), ("_theorem_m64", fa)):
            cases[f"cp_r10{rname}_{prec}"] = (prec, lambda ff=ff, prec=prec: ctx.apply_cp(ff, U, prec=prec))
            cases[f"tucker_888{rname}_{prec}"] = (prec, lambda ff=ff, prec=prec: ctx.apply_tucker(ff, V, prec=prec))
            cases[f"tt_188_1{rname}_{prec}"] = (prec, lambda ff=ff, prec=prec: ctx.apply_tt(ff, G1, G2, G3, prec=prec))
    for name, (prec, fn) in cases.items():
        ms, prof = _timed(ctx, fn, args.steps, args.warmup)
        rec = prof["fft/xyz" if prec == "fp64" else "fft32/xyz"]
        per_ms = rec["ms"] / rec["launches"]
        bytes_ = rec["bytes"] / rec["launches"]
        flops = rec["flops"] / rec["launches"]
        achieved = bytes_ / (per_ms * 1e-3) / 1e9
        out[name] = {"ms_per_apply": round(ms, 4), "implicit_cells_per_s": n ** 3 / (ms * 1e-3), "transforms": prec,
                     "roofline": {"bound": "hbm", "kernel": "k_fft_fwd + k_fft_jobs (one apply)",
                                  "achieved": round(achieved, 1), "peak": HBM_GBS, "unit": "GB/s",
                                  "frac": round(achieved / HBM_GBS, 4), "traffic": None,
                                  "algorithmic_bytes_per_launch": bytes_, "avg_launch_ms": round(per_ms, 4)},
                     "fft_gflops": round(flops / (per_ms * 1e-3) / 1e9, 1), "kernels": _kernels(prof, args.steps)}
        # the same launches against the vector-ALU peak of the transform
        # precision (flops: 2.5 L log2 L per real transform of length L);
        # FP32's published peak counts packed FP32, which this build does not
        # issue, so half of it is the reachable ceiling there
        tflops = flops / (per_ms * 1e-3) / 1e12
        vpeak = FP64_VEC_TFLOPS if prec == "fp64" else FP32_VEC_TFLOPS
        out[name]["valu"] = {"achieved": round(tflops, 2), "peak": vpeak, "unit": "TFLOP/s",
                             "frac": round(tflops / vpeak, 4),
                             "frac_unpacked": round(tflops / FP64_VEC_TFLOPS, 4) if prec == "fp32" else None}
    # HOOI recompression of the CP apply's potential (3 M r terms) to Tucker
    # form, for the random rank-10 input above and a smooth one
    recomp = {}
    x = np.linspace(0.0, 1.0, n)
    rng = np.random.default_rng(9)
    smooth = [np.stack([np.stack([np.cos(np.pi * (l + 1) * rng.uniform(0.5, 1.5) * x + rng.uniform(0, 3))
                                  for l in range(10)]) for _q in range(3)]).astype(np.float32) for _d in range(3)]
    for name, cols_in in (("cp_r10_random", U), ("cp_r10_smooth", [torch.from_numpy(c).cuda() for c in smooth])
                          ) if args.recompress else ():
        out_cols, table = ctx.apply_cp(f, cols_in)
        T = table.shape[1]
        tab = torch.from_numpy(np.ascontiguousarray(table[0])).cuda()
        lam = torch.ones(T, dtype=torch.float64, device="cuda")
        for eps in (1e-3, 1e-6):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.recompress_cp((n, n, n), out_cols, tab, lam, eps, rmax=64, max_sweeps=10)
            sec = time.perf_counter() - t0
            recomp[f"{name}_eps{eps:g}"] = {"terms": T, "ranks": res["ranks"], "rel_err": res["rel_err"],
                                           "sweeps": res["sweeps"], "seconds": round(sec, 4),
                                           "tolerance_met": res["rel_err"] <= eps}
        del out_cols
    del U, V, G1, G2, G3, f, fa
    torch.cuda.empty_cache()
    return {"workload": "structured apply, n=4096 per axis, CP rank 10 / Tucker (8,8,8) / TT (1,8,8,1), U[-1,1] "
                        "factors seed 1; sinc rule M=40 (c0=2.15) and the theorem-step rule with 64 nodes; FP32 "
                        "columns; FP64 transforms, and FP32 transforms (FP64 forward transforms of the inputs)",
            "certified_rule_err": {k: {"phi": v[0], "h": v[1]} for k, v in certified.items()},
            "results": out, "recompression_phi": recomp}


def tucker_record(ctx, args):
    """Alg. scpot_fft_tucker (structured DFTs with tolerance-controlled
    Tucker arithmetic): the paper's uniform-magnetization case on cubes of
    n = 256, 1024, 4096 cells per axis, and a smooth rank-(2,2,2)
    magnetization at n = 4096; M = 40 (c0 = 2.15), tol 1e-8.  Wall times of
    the set-up (kernel compression and DFTs) and of one potential (the loop
    and the approximate summation; median of 3), with the ranks."""
    import torch

    from paper_1212_3509_amd import inputs

    def dev(t):
        core, U = t
        return (torch.from_numpy(core.copy()).cuda(), [torch.from_numpy(U[p].T.copy()).cuda() for p in range(3)])

    out = {"workload": "Alg. scpot_fft_tucker, uniform magnetization (0.3, -0.5, 0.8) on n^3 cubes and a smooth "
                       "rank-(2,2,2) magnetization at n = 4096, M = 40 (c0 = 2.15), tol 1e-8, FP64",
           "cases": []}
    for n, kind in ((256, "uniform"), (1024, "uniform"), (4096, "uniform"), (4096, "smooth")):
        nn = (n, n, n)
        f = ctx.assemble(nn, (1.0 / n,) * 3, M=40)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kt = ctx.ktucker(f, 1e-8)
        setup = time.perf_counter() - t0
        mag = [dev(t) for t in inputs.tucker_magnetization(nn, kind, (2, 2, 2))]
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            core, rows = ctx.potential_tucker(kt, mag, 1e-8)
            times.append(time.perf_counter() - t0)
        out["cases"].append({"n": n, "input": kind, "kernel_ranks": [list(kt.ranks(q)) for q in range(3)],
                             "potential_ranks": list(core.shape), "setup_ms": round(setup * 1e3, 2),
                             "potential_ms": round(sorted(times)[1] * 1e3, 2)})
        kt.close()
        f.free()
    return out


def structured(args):
    from paper_1212_3509_amd import api
    if args.calib_copy_mib > 0:
        _copy_calibration(args.calib_copy_mib)
    print(json.dumps({"n_gpus": 1, **structured_record(api.Context(0), args)}), flush=True)


def tucker(args):
    from paper_1212_3509_amd import api
    print(json.dumps({"n_gpus": 1, **tucker_record(api.Context(0), args)}), flush=True)


def batch_record(args):
    """256 magnetization states on uneven grids, FP32, one persistent launch
    per stage, graph replay, autotuned tiles; roofline on the FP32 matrix
    cores (algorithmic FLOPs of the dense Toeplitz products)."""
    import numpy as np
    import torch

    from paper_1212_3509_amd import api, inputs

    states = inputs.batch_grids(256, seed=2, with_fields=True)
    ctx = api.Context(0)
    ctx.set_workspace_limit(int(args.batch_ws_gib) << 30)
    b = ctx.batch([(s.n, s.h) for s in states], M=40, prec="fp32")
    t0 = time.perf_counter()
    if args.tune:
        b.tune(args.tune_cache or None, reps=2)
    tune_s = time.perf_counter() - t0
    off = b.offsets()
    m = torch.from_numpy(np.concatenate([s.m.reshape(-1) for s in states]).astype(np.float32)).cuda()
    phi = torch.empty(int(off[-1]), dtype=torch.float32, device="cuda")
    h = torch.empty(3 * int(off[-1]), dtype=torch.float32, device="cuda")
    ms, prof = _timed(ctx, lambda: b.apply(m, phi, h, use_graph=True), args.steps, args.warmup)
    info = b.info()
    achieved = info["flops"] / (ms * 1e-3) / 1e12
    rec = {"workload": "256 states on uneven grids (cubes 16..96, films 256x256x{4,8,16}, seed 2), FP32, M=40, "
                       "one persistent launch per stage, graph replay",
           "cells": int(off[-1]), "ms_per_batch": round(ms, 3), "Mcell_per_s": round(off[-1] / (ms * 1e-3) / 1e6, 2),
           "roofline": {"bound": "mfma", "kernel": "k_left_items (all stages of one batch)",
                        "achieved": round(achieved, 2), "peak": PEAK_TFLOPS["fp32"], "unit": "TFLOP/s",
                        "frac": round(achieved / PEAK_TFLOPS["fp32"], 4), "traffic": None,
                        "flops_per_batch": info["flops"]},
           "tune_seconds": round(tune_s, 2), "node_chunk": info["node_chunk"],
           "persistent_groups": info["persistent_groups"]}
    del m, phi, h, b, ctx
    torch.cuda.empty_cache()
    return rec


def batch(args):
    print(json.dumps({"n_gpus": 1, **batch_record(args)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="headline", choices=["headline", "cp4096", "batch", "tucker"])
    ap.add_argument("--cpu-runs", type=int, default=3, help="runs (median) of each CPU baseline timing (0: skip)")
    ap.add_argument("--precs", default="fp64,fp32,bf16x3,bf16x2")
    ap.add_argument("--learned-steps", type=int, default=4000)
    ap.add_argument("--fit-iters", type=int, default=60, help="LM iterations of the training fits")
    ap.add_argument("--predict-iters", type=int, default=200, help="LM iterations per fit in predict")
    ap.add_argument("--structured", type=int, default=1, help="also time the structured applies at n = 4096")
    ap.add_argument("--batch", type=int, default=1, help="also time the batch of 256 uneven states")
    ap.add_argument("--tucker", type=int, default=1, help="also time the Tucker DFT route (Alg. scpot_fft_tucker)")
    ap.add_argument("--cases", type=int, default=20000)
    ap.add_argument("--rule-tol", type=float, default=1e-6)
    ap.add_argument("--mixed-prec", default="bf16x3")
    ap.add_argument("--batch-ws-gib", type=int, default=64)
    ap.add_argument("--tune", type=int, default=1)
    ap.add_argument("--tune-cache", default="", help="batch: JSON file of tuned tile shapes to read and extend")
    ap.add_argument("--fft3d", type=int, default=1, help="also time the 3D-FFT route of the same operator")
    ap.add_argument("--nonuniform", type=int, default=1, help="also time the apply on a graded non-uniform grid")
    ap.add_argument("--learned-eval", type=int, default=1,
                    help="evaluate the trained network at 256^3 full format and 1024^3 CP rank 10")
    ap.add_argument("--recompress", type=int, default=1, help="cp4096: also time the HOOI recompression")
    ap.add_argument("--vendor-gemm", type=int, default=1,
                    help="also time torch.matmul at FP64/FP32/BF16 as context for the matrix-core figures")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain copy of this many MiB first (byte-counter calibration)")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU work: rewrite the HBM counter summary from two rocprofv3 --pmc CSVs "
                         "(with --calib-copy-mib of the profiled run)")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(*args.write_traffic, args.calib_copy_mib)
        return
    if args.gpus != 1:
        print("bench.py: this library runs on a single GPU; multi-GPU runs (sharding the quadrature nodes, "
              "states or structured jobs over ranks) are not implemented", file=sys.stderr)
        sys.exit(2)
    {"headline": headline, "cp4096": structured, "batch": batch, "tucker": tucker}[args.workload](args)


if __name__ == "__main__":
    main()
