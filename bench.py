#!/usr/bin/env python3
"""Bench of the H-matrix Helmholtz single-layer operator on one MI355X.

Workload (synthetic, seeded): unit icosphere with 81 920 triangles (6 refinements), 3-point
interior rule (245 760 points), Helmholtz k = 40, cluster leaf 64, admissibility eta = 1.5, ACA
tolerance 1e-3, complex N(0,1) vector with seed 0.  One step = one full pass of the hot path:
quadrature points, cluster tree, block tree, near-field blocks, ACA of the far blocks, and one
H-matrix product, with the mesh and the vector already resident in device memory.

Printed JSON line: the step time, the build and product times, the relative error on seeded
sampled rows against the CPU oracle's dense product, the roofline of the product kernels, and the
CPU oracle's own build + product time on the host cores (the cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H-matvec ms and H-build s at 1e-3 rel err; kernel evals/s; frac of HBM/FP peak"
HBM_PEAK_GBS = 8000.0
ACA_BIG_KERNEL = "hmx::aca_kernel<T, 512> (ACA of the far blocks with m + n >= 4096)"
PMC_SUMMARY = {"fp64": os.path.join(ROOT, "profiles", "aca_big_icosphere_L6_k40_fp64_pmc.txt"),
               "fp32": os.path.join(ROOT, "profiles", "aca_big_icosphere_L6_k40_fp32_pmc.txt")}
ACA_SOURCE = os.path.join(ROOT, "paper_1804_00995_amd", "csrc", "k_aca.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest(path):
    import hashlib
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(precision):
    """HBM bytes per launch of the large-block ACA kernel from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None when the summary
    is missing or the kernel source has changed since the counters were taken."""
    path = PMC_SUMMARY[precision]
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                key, _, val = line.partition(":")
                vals[key.strip()] = val.strip()
    if vals.get("k_aca.hip sha256[:16]") != source_digest(ACA_SOURCE):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain elementwise copy (torch.neg into a second buffer) of known size, for scaling the
    FETCH_SIZE / WRITE_SIZE counters: reads and writes mib MiB per launch, 5 launches."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": n * 8,
                                           "bytes_written_per_launch": n * 8, "launches": 5}}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--level", type=int, default=6)
    ap.add_argument("--k", type=float, default=40.0)
    ap.add_argument("--matvec-reps", type=int, default=30)
    ap.add_argument("--sample-rows", type=int, default=384)
    ap.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run the copy kernel used to scale the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        log("bench.py measures a single GPU; --gpus above 1 is not supported")
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return

    import torch

    import oracle
    from paper_1804_00995_amd import hmx
    from paper_1804_00995_amd import inputs as I

    dev = torch.device("cuda:0")
    v, f = I.icosphere(args.level)
    bary, w = I.rule_3pt()
    M = 3 * f.shape[0]
    prec = hmx.FP64 if args.precision == "fp64" else hmx.FP32_MIXED
    cdt = torch.complex128 if prec == hmx.FP64 else torch.complex64
    prm = hmx.params(tol=1e-3, leaf_size=64, eta=1.5, precision=prec)
    x_h = I.complex_vector(M, 0)
    vd = torch.from_numpy(v).to(dev)
    fd = torch.from_numpy(f).to(dev)
    xd = torch.from_numpy(x_h).to(cdt).to(dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    log(f"bench: M={M} k={args.k} precision={args.precision} steps={args.steps} warmup={args.warmup}")

    def step():
        op = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=args.k, prm=prm, stream=stream)
        y = op.matvec(xd, stream=stream)
        return op, y

    for i in range(args.warmup):
        op, y = step()
        torch.cuda.synchronize()
        op.close()
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    aca = []  # per timed step: (ms, algorithmic bytes, rounds) of the large-block ACA launch
    t0 = time.perf_counter()
    for i in range(args.steps):
        op, y = step()
        aca.append((op.info["aca_ms"][0], op.info["aca_bytes"][0], op.info["aca_rounds"]))
        op.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / max(args.steps, 1)
    log(f"timed steps done: {ms_step:.1f} ms/step")

    # product timing and accuracy on one more operator (outside the timed region)
    op, y = step()
    torch.cuda.synchronize()
    info = op.info
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(args.matvec_reps):
        ev0.record(stream)
        op.matvec(xd, y, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    mv_ms = float(np.median(times))
    log(f"matvec {mv_ms:.3f} ms (median of {args.matvec_reps})")
    y_h = y.cpu().numpy().astype(np.complex128)
    P, Wq = oracle.quad_points(v, f, bary, w)
    rows = np.sort(np.random.default_rng(123).choice(M, args.sample_rows, replace=False))
    yr = oracle.dense_rows(P, Wq, oracle.HELMHOLTZ, args.k, x_h, rows)
    rel_err = float(np.linalg.norm(y_h[rows] - yr) / np.linalg.norm(yr))
    log(f"rel_err on {args.sample_rows} sampled rows: {rel_err:.3e}")

    elem = 16 if prec == hmx.FP64 else 8
    stored = info["near_entries"] + info["far_entries"] + info["dense_far_entries"]
    mv_bytes = elem * (stored + 4 * M) + 8 * M
    mv_achieved = mv_bytes / (mv_ms * 1e-3) / 1e9
    build_s = info["t_total_ms"] / 1e3
    # dominant kernel of the step: ACA of the large far blocks (one launch per build)
    aca_ms = float(np.mean([a[0] for a in aca])) if aca else info["aca_ms"][0]
    aca_bytes = aca[-1][1] if aca else info["aca_bytes"][0]
    aca_gbs = aca_bytes / (aca_ms * 1e-3) / 1e9 if aca_ms > 0 else 0.0
    traffic = measured_traffic(args.precision)

    cpu = None
    if args.cpu_baseline == "on":
        log("cpu baseline: oracle H-build + H-matvec on the host cores")
        c0 = time.perf_counter()
        Ho = oracle.HMatrix(P, Wq, oracle.HELMHOLTZ, args.k, leaf=64, eta=1.5, tol=1e-3)
        c1 = time.perf_counter()
        Ho.matvec(x_h)
        c2 = time.perf_counter()
        Ho.close()
        cpu = {"value": round((c2 - c0) * 1e3, 1), "unit": "ms per step (H-build + one H-matvec)",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"full workload once: build {c1 - c0:.2f} s, product {c2 - c1:.2f} s"}
        log(f"cpu baseline {cpu}")

    out = {
        "metric": METRIC,
        "value": round(ms_step, 3),
        "unit": "ms per step (H-build from device mesh + one H-matvec)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == hmx.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"unit icosphere L{args.level} ({f.shape[0]} triangles, {M} points), "
                               f"Helmholtz k={args.k:g}, leaf 64, eta 1.5, ACA tol 1e-3, "
                               f"{args.precision}"},
        "h_build_s": round(build_s, 4),
        "h_matvec_ms": round(mv_ms, 4),
        "rel_err": rel_err,
        "kernel_evals_per_s": info["kernel_evals"] / build_s if build_s > 0 else None,
        "build_phases_ms": {k2: round(info[k2], 2) for k2 in
                            ("t_tree_ms", "t_blocks_ms", "t_near_ms", "t_aca_ms")},
        "sizes": {k2: info[k2] for k2 in ("n_near", "n_far", "near_entries", "far_entries",
                                           "dense_far", "max_rank", "overflow_blocks", "bytes")},
        "roofline": {"bound": "hbm", "kernel": ACA_BIG_KERNEL, "achieved": round(aca_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(aca_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "launch_ms": round(aca_ms, 3),
                     "algorithmic_bytes_per_launch": aca_bytes,
                     "blocks": info["aca_blocks"][0], "rounds": max(a[2] for a in aca) if aca else None},
        "roofline_matvec": {"bound": "hbm", "achieved": round(mv_achieved, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(mv_achieved / HBM_PEAK_GBS, 4),
                            "bytes_per_product": mv_bytes},
        "aca_classes": {"blocks": info["aca_blocks"], "first_launch_ms": [round(t, 3) for t in info["aca_ms"]],
                        "algorithmic_bytes": info["aca_bytes"]},
        "cpu_baseline": cpu,
    }
    op.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
