#!/usr/bin/env python3
"""Bench of the H-matrix Helmholtz single-layer operator on one MI355X.

Workloads (synthetic, seeded), selected with --workload:
  sphere (default)  unit icosphere with 81 920 triangles (6 refinements), 3-point interior rule
                    (245 760 points), Helmholtz k = 40, cluster leaf 64, admissibility
                    eta = 1.5, ACA tolerance 1e-3, complex N(0,1) vector with seed 0;
  batch             64 seeded ellipsoids (semi-axes U[0.5, 2], 2 000-40 000 triangles
                    log-uniform, k U[2, 30], vector seed 1000 + i) built and applied as one
                    block-diagonal operator;
  target            the same batch in FP32 mixed precision with the learned rank layout (network
                    trained on the sphere workload's FP64 and FP32 ranks) and the autotuned batch
                    schedule, reported against the plain FP64 batch;
  large             one eighth (row share 0 of 8) of the prolate (2, 1, 1) ellipsoid with
                    1 310 720 triangles (3 932 160 points), k = 120, leaf 128, tol 1e-4, FP32;
                    100 products replayed in one HIP graph; --large-shares all: the whole
                    operator as its 8 row shares built and applied in turn.
One step = one full pass of the hot path with the mesh and the vector already resident in device
memory: quadrature points, cluster tree, block tree, near-field blocks, ACA of the far blocks,
and one H-matrix product.

Printed JSON line: the step time, the build and product times, the relative error on seeded
sampled rows against the CPU oracle's dense product, the roofline of the dominant kernel (ACA of
the large far blocks, timed by events inside the library on its own stream), the roofline of the
product, and the CPU oracle timed on the host cores (cpu_baseline).
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
ACA_BIG_KERNEL = "hmx::aca_kernel<T, NT, true> (ACA of the far blocks with m + n >= 4096; NT = 512 for FP64, 256 for FP32)"
PMC_SUMMARY = {"fp64": os.path.join(ROOT, "profiles", "aca_big_icosphere_L6_k40_fp64_pmc.txt"),
               "fp32": os.path.join(ROOT, "profiles", "aca_big_icosphere_L6_k40_fp32_pmc.txt")}
# the large-block ACA kernel's source and the headers it includes: the counter summary's traffic
# is used only while all of them are unchanged
ACA_SOURCES = tuple(os.path.join(ROOT, "paper_1804_00995_amd", "csrc", f)
                    for f in ("k_aca.hip", "hmx_dev.h", "hmx_host.h"))
DIGEST_KEY = "aca sources sha256[:16]"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest(*paths):
    import hashlib
    h = hashlib.sha256()
    for path in paths:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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
            if ": " in line and not line.startswith(" "):
                key, _, val = line.partition(": ")  # keys may hold a colon ("sha256[:16]")
                vals[key.strip()] = val.strip()
    if vals.get(DIGEST_KEY) != source_digest(*ACA_SOURCES):
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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    times = []
    for _ in range(5):
        ev[0].record()
        torch.neg(a, out=b)
        ev[1].record()
        ev[1].synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    torch.cuda.synchronize()
    ms = float(np.median(times))
    print(json.dumps({"copy_calibration": {"bytes_read_per_launch": n * 8,
                                           "bytes_written_per_launch": n * 8, "launches": 5,
                                           "median_ms": round(ms, 4),
                                           "gb_per_s": round(2 * n * 8 / (ms * 1e-3) / 1e9, 1)}}))


def timed_steps(step, steps, warmup):
    """Run `warmup` untimed and `steps` timed steps (synchronised on both sides); returns the
    ms per step and, per timed step, (large-block ACA launch ms, its algorithmic bytes, rounds)."""
    import torch
    for i in range(warmup):
        op, _ = step()
        torch.cuda.synchronize()
        op.close()
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    aca = []
    t0 = time.perf_counter()
    for _ in range(steps):
        op, _ = step()
        aca.append((op.info["aca_ms"][0], op.info["aca_bytes"][0], op.info["aca_rounds"]))
        op.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / max(steps, 1)
    log(f"timed steps done: {ms:.1f} ms/step")
    return ms, aca


def product_ms(op, xd, y, stream, reps):
    import torch
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(reps):
        ev0.record(stream)
        op.matvec(xd, y, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    return float(np.median(times))


def rooflines(info, aca, mv_ms, M, elem, precision, near_stored=True):
    # bytes a product reads: the stored entries (the near blocks only when stored) and vectors
    stored = (info["near_entries"] if near_stored else 0) + info["far_entries"] + info["dense_far_entries"]
    mv_bytes = elem * (stored + 4 * M) + 8 * M
    mv_gbs = mv_bytes / (mv_ms * 1e-3) / 1e9
    aca_ms = float(np.mean([a[0] for a in aca])) if aca else info["aca_ms"][0]
    aca_bytes = aca[-1][1] if aca else info["aca_bytes"][0]
    aca_gbs = aca_bytes / (aca_ms * 1e-3) / 1e9 if aca_ms > 0 else 0.0
    return {
        "roofline": {"bound": "hbm", "kernel": ACA_BIG_KERNEL, "achieved": round(aca_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(aca_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(precision), "launch_ms": round(aca_ms, 3),
                     "algorithmic_bytes_per_launch": aca_bytes, "blocks": info["aca_blocks"][0],
                     "rounds": max(a[2] for a in aca) if aca else None},
        "roofline_matvec": {"bound": "hbm", "achieved": round(mv_gbs, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(mv_gbs / HBM_PEAK_GBS, 4),
                            "bytes_per_product": mv_bytes},
        "aca_classes": {"order": ["large (m + n >= aca_big_mn)", "middle", "wavefront (m, n <= 64)",
                                  "small (m + n < aca_small_mn)"],
                        "blocks": info["aca_blocks"],
                        "first_launch_ms": [round(t, 3) for t in info["aca_ms"]],
                        "algorithmic_bytes": info["aca_bytes"],
                        "algorithmic_gb_per_s": [round(b / (t * 1e-3) / 1e9, 1) if t > 0 and b > 0 else None
                                                 for b, t in zip(info["aca_bytes"], info["aca_ms"])],
                        "frac_of_peak": [round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if t > 0 and b > 0 else None
                                         for b, t in zip(info["aca_bytes"], info["aca_ms"])]},
    }


def sizes(info):
    return {k2: info[k2] for k2 in ("n_near", "n_far", "near_entries", "far_entries", "dense_far",
                                     "max_rank", "overflow_blocks", "bytes", "factor_bytes")}


def line(args, ms_step, prec_name, config, extra,
         unit="ms per step (H-build from device mesh + one H-matvec)"):
    out = {
        "metric": METRIC,
        "value": round(ms_step, 3),
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_name == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": config,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------------------- workloads
def run_sphere(args, torch, oracle, hmx, I):
    dev = torch.device("cuda:0")
    v, f = I.icosphere(args.level)
    bary, w = I.rule_3pt()
    M = 3 * f.shape[0]
    prec = hmx.FP64 if args.precision == "fp64" else hmx.FP32_MIXED
    cdt = torch.complex128 if prec == hmx.FP64 else torch.complex64
    reg = args.regularize == "on"
    prm = hmx.params(tol=1e-3, leaf_size=64, eta=1.5, precision=prec, regularize=int(reg),
                     aca_serial=int(args.aca_serial == "on"),
                     near_mode=int(args.near_mode == "otf" and not reg))  # (the correction
    # lives in stored near blocks)
    x_h = I.complex_vector(M, 0)
    vd, fd = torch.from_numpy(v).to(dev), torch.from_numpy(f).to(dev)
    xd = torch.from_numpy(x_h).to(cdt).to(dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    log(f"bench sphere: M={M} k={args.k} precision={args.precision} singular correction={reg}")

    def step():
        op = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=args.k, prm=prm, stream=stream)
        return op, op.matvec(xd, stream=stream)

    ms_step, aca = timed_steps(step, args.steps, args.warmup)
    op, y = step()  # product timing and accuracy on one more operator (outside the timed region)
    torch.cuda.synchronize()
    info = op.info
    mv_ms = product_ms(op, xd, y, stream, args.matvec_reps)
    log(f"matvec {mv_ms:.3f} ms (median of {args.matvec_reps})")
    # several vectors at once: ms per vector of hmx_matvec_multi (groups of four read the
    # operator once), to show where the per-vector cost stops falling
    multi = {}
    if args.multi_vectors > 1:
        for nr in (2, 4, 8, 16):
            if nr > args.multi_vectors:
                break
            X = xd.unsqueeze(0).repeat(nr, 1).contiguous()
            Y = torch.empty_like(X)
            op.matvec_multi(X, Y, stream=stream)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            times = []
            for _ in range(5):
                ev0.record(stream)
                op.matvec_multi(X, Y, stream=stream)
                ev1.record(stream)
                ev1.synchronize()
                times.append(ev0.elapsed_time(ev1))
            multi[str(nr)] = round(float(np.median(times)) / nr, 4)
        multi["1"] = round(mv_ms, 4)
        log(f"ms per vector, several-vector product: {multi}")
    y_h = y.cpu().numpy().astype(np.complex128)
    build_s = info["t_total_ms"] / 1e3
    cpu, rel_err = None, None
    if args.cpu_baseline == "on":
        # the oracle leg: the error of the GPU product on sampled rows, then the oracle timed
        P, Wq = oracle.quad_points(v, f, bary, w)
        rows = np.sort(np.random.default_rng(123).choice(M, args.sample_rows, replace=False))
        yr = oracle.dense_rows(P, Wq, oracle.HELMHOLTZ, args.k, x_h, rows)
        if reg:  # the corrected dense rows: every close pair's correction on top
            yr = yr + oracle.reg_apply(P, Wq, v, f, bary, 2.0, x_h, rows=rows)
        rel_err = float(np.linalg.norm(y_h[rows] - yr) / np.linalg.norm(yr))
        log(f"rel_err on {args.sample_rows} sampled rows: {rel_err:.3e}")
        log("cpu baseline: oracle H-build + H-matvec on the host cores")
        c0 = time.perf_counter()
        Ho = oracle.HMatrix(P, Wq, oracle.HELMHOLTZ, args.k, leaf=64, eta=1.5, tol=1e-3,
                            mesh=(v, f, bary) if reg else None)
        c1 = time.perf_counter()
        Ho.matvec(x_h)
        c2 = time.perf_counter()
        Ho.close()
        cores = oracle.max_threads()
        cpu = {"value": round((c2 - c0) * 1e3, 1), "unit": "ms per step (H-build + one H-matvec)",
               "cores": cores, "kind": "oracle",
               "sample": f"full workload once: build {c1 - c0:.2f} s, product {c2 - c1:.2f} s "
                         f"(both on {cores} threads)"}
        if args.cpu_one_core == "on":
            # the same oracle on one core, beside the paper's single-core timings
            c0 = time.perf_counter()
            Ho = oracle.HMatrix(P, Wq, oracle.HELMHOLTZ, args.k, leaf=64, eta=1.5, tol=1e-3,
                                mesh=(v, f, bary) if reg else None, nthreads=1)
            c1 = time.perf_counter()
            Ho.matvec(x_h)
            c2 = time.perf_counter()
            Ho.close()
            oracle.HMatrix(P[:8], Wq[:8], oracle.LAPLACE, 0.0, leaf=64, nthreads=cores).close()
            cpu["one_core"] = {"build_s": round(c1 - c0, 2), "product_s": round(c2 - c1, 3)}
        log(f"cpu baseline {cpu}")
    extra = {
        "h_build_s": round(build_s, 4),
        "h_matvec_ms": round(mv_ms, 4),
        "rel_err": rel_err,
        "kernel_evals_per_s": info["kernel_evals"] / build_s if build_s > 0 else None,
        "build_phases_ms": {k2: round(info[k2], 2) for k2 in
                            ("t_tree_ms", "t_blocks_ms", "t_near_ms", "t_aca_ms")},
        "sizes": sizes(info),
    }
    extra.update(rooflines(info, aca, mv_ms, M, 16 if prec == hmx.FP64 else 8, args.precision,
                           near_stored=prm.near_mode == 0))
    if args.aca_serial != "on":
        # each ACA class on its own: one more build (untimed) with the classes one after the
        # other, whose first launches are then each class's own duration (concurrent, a class's
        # launch also spans the time it waits for room beside the others)
        ops = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=args.k, stream=stream,
                        prm=hmx.params(tol=1e-3, leaf_size=64, eta=1.5, precision=prec,
                                       regularize=int(reg), aca_serial=1,
                                       near_mode=prm.near_mode))
        alone = list(ops.info["aca_ms"])
        ops.close()
        cls = extra["aca_classes"]
        cls["alone_ms"] = [round(t, 3) for t in alone]
        cls["alone_frac_of_peak"] = [round(b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if t > 0 and b > 0
                                     else None for b, t in zip(cls["algorithmic_bytes"], alone)]
        log(f"ACA classes one at a time: {cls['alone_ms']} ms")
    # kernel evaluations per second by phase: near-field assembly (its phase time includes the
    # block bookkeeping; none when the product computes the near field), and ACA rows and
    # columns; the ALU ceiling of one evaluation beside them
    near_s, aca_s = info["t_near_ms"] / 1e3, info["t_aca_ms"] / 1e3
    near_built = info["near_entries"] if prm.near_mode == 0 else 0
    extra["evals_per_s"] = {
        "near_assembly": near_built / near_s if near_built and near_s > 0 else None,
        "aca_rows_columns": (info["kernel_evals"] - near_built) / aca_s if aca_s > 0 else None,
        "alu_ceiling": DENSE_ALU_PEAK[args.precision],
    }
    if multi:
        extra["ms_per_vector_several"] = multi
    extra["cpu_baseline"] = cpu
    op.close()
    config = {"workload": f"unit icosphere L{args.level} ({f.shape[0]} triangles, {M} points), "
                          f"Helmholtz k={args.k:g}, leaf 64, eta 1.5, ACA tol 1e-3, {args.precision}"
                          + (", singular correction (radius 2)" if reg else "")
                          + (", near field computed in the product"
                             if args.near_mode == "otf" and not reg else "")}
    line(args, ms_step, args.precision, config, extra)


def batch_errors(oracle, meshes, descs, bary, w, x_h, y_h, off, rows_per_mesh=24, seed=77):
    """Relative errors of a batch product on seeded sampled rows of every mesh against the
    oracle's dense rows: (all sampled rows together, worst mesh)."""
    rng = np.random.default_rng(seed)
    errs, num, den = [], 0.0, 0.0
    for i, ((v, f), d) in enumerate(zip(meshes, descs)):
        P, Wq = oracle.quad_points(v, f, bary, w)
        rows = np.sort(rng.choice(P.shape[0], rows_per_mesh, replace=False))
        yr = oracle.dense_rows(P, Wq, oracle.HELMHOLTZ, d["k"], x_h[off[i]:off[i + 1]], rows)
        diff = np.linalg.norm(y_h[off[i] + rows] - yr)
        errs.append(float(diff / np.linalg.norm(yr)))
        num += diff ** 2
        den += np.linalg.norm(yr) ** 2
    return float(np.sqrt(num / den)), max(errs)


def run_batch(args, torch, oracle, hmx, I):
    descs = I.batch_ellipsoids(64, seed=0)
    bary, w = I.rule_3pt()
    prec = hmx.FP64 if args.precision == "fp64" else hmx.FP32_MIXED
    cdt = torch.complex128 if prec == hmx.FP64 else torch.complex64
    prm = hmx.params(tol=1e-3, leaf_size=64, eta=1.5, precision=prec,
                     near_mode=int(args.near_mode == "otf"))
    meshes, dev = [], []
    for d in descs:
        v, f = I.batch_mesh(d)
        meshes.append((v, f))
        dev.append((torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), d["k"]))
    x_h = np.concatenate([I.complex_vector(3 * f.shape[0], d["seed"]) for d, (_, f) in zip(descs, meshes)])
    M = x_h.shape[0]
    xd = torch.from_numpy(x_h).to(cdt).cuda()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    log(f"bench batch: 64 meshes, {M} points, precision={args.precision}")

    def step():
        op = hmx.build_batch(dev, bary, w, kern=hmx.HELMHOLTZ, prm=prm, stream=stream)
        return op, op.matvec(xd, stream=stream)

    ms_step, aca = timed_steps(step, args.steps, args.warmup)
    op, y = step()
    torch.cuda.synchronize()
    info = op.info
    mv_ms = product_ms(op, xd, y, stream, args.matvec_reps)
    off = op.mesh_offsets()
    y_h = y.cpu().numpy().astype(np.complex128)
    cpu, rel_err, rel_err_worst = None, None, None
    if args.cpu_baseline == "on":
        # the oracle leg: errors of the GPU product on sampled rows of every mesh
        rel_err, rel_err_worst = batch_errors(oracle, meshes, descs, bary, w, x_h, y_h, off)
        log(f"batch errors: worst mesh {rel_err_worst:.3e}, all sampled rows {rel_err:.3e}")
        # bounded sample: the oracle H-build + product of the first 8 meshes, scaled by points
        c0 = time.perf_counter()
        m_sample = 0
        for (v, f), d in list(zip(meshes, descs))[:8]:
            P, Wq = oracle.quad_points(v, f, bary, w)
            Ho = oracle.HMatrix(P, Wq, oracle.HELMHOLTZ, d["k"], leaf=64, eta=1.5, tol=1e-3)
            Ho.matvec(I.complex_vector(P.shape[0], d["seed"]))
            Ho.close()
            m_sample += P.shape[0]
        c1 = time.perf_counter()
        cpu = {"value": round((c1 - c0) * 1e3 * M / m_sample, 1),
               "unit": "ms per step (H-build + one H-matvec), scaled by points",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"first 8 of the 64 meshes ({m_sample} of {M} points) in {c1 - c0:.2f} s, "
                         "scaled linearly by points"}
    build_s = info["t_total_ms"] / 1e3
    extra = {
        "h_build_s": round(build_s, 4),
        "h_matvec_ms": round(mv_ms, 4),
        "rel_err": rel_err,
        "rel_err_worst_mesh": rel_err_worst,
        "kernel_evals_per_s": info["kernel_evals"] / build_s if build_s > 0 else None,
        "build_phases_ms": {k2: round(info[k2], 2) for k2 in
                            ("t_tree_ms", "t_blocks_ms", "t_near_ms", "t_aca_ms")},
        "sizes": sizes(info),
    }
    extra.update(rooflines(info, aca, mv_ms, M, 16 if prec == hmx.FP64 else 8, args.precision,
                           near_stored=prm.near_mode == 0))
    extra["roofline"]["traffic"] = None  # counters were taken on the sphere workload
    extra["cpu_baseline"] = cpu
    op.close()
    config = {"workload": f"64 seeded ellipsoids ({M} points), Helmholtz k U[2,30], leaf 64, "
                          f"eta 1.5, ACA tol 1e-3, one block-diagonal operator, {args.precision}"
                          + (", near field computed in the product" if prm.near_mode else "")}
    line(args, ms_step, args.precision, config, extra)


def run_target(args, torch, oracle, hmx, I):
    """The batch of 64 ellipsoids in its target form -- FP32 mixed precision, the learned
    rank layout from a network trained on the 245 760-point sphere's ranks (k = 40, FP64 and
    FP32 builds; the ellipsoids are never seen in training) and the batch schedule picked by
    the autotuner -- against the plain FP64 batch (adaptive ACA, default schedule)."""
    from paper_1804_00995_amd import rank_model as R
    bary, w = I.rule_3pt()
    # training data: far-block features and ranks of the sphere workload in both precisions
    vs, fs = I.icosphere(6)
    vsd, fsd = torch.from_numpy(vs).cuda(), torch.from_numpy(fs).cuda()
    feats, ranks = [], []
    for prec in (hmx.FP64, hmx.FP32_MIXED):
        op = hmx.build(vsd, fsd, bary, w, kern=hmx.HELMHOLTZ, k=40.0,
                       prm=hmx.params(tol=1e-3, leaf_size=64, eta=1.5, precision=prec))
        f_, r_ = R.block_data(op)
        feats.append(f_)
        ranks.append(r_)
        op.close()
    t0 = time.perf_counter()
    model = R.train(np.concatenate(feats), np.concatenate(ranks), epochs=args.train_epochs)
    train_s = time.perf_counter() - t0
    log(f"rank model: {sum(len(r) for r in ranks)} sphere blocks, {args.train_epochs} epochs in "
        f"{train_s:.1f} s, alpha {model.alpha:.3f}, final loss {model.history[-1]:.4f}")

    descs = I.batch_ellipsoids(64, seed=0)
    meshes, dev = [], []
    for d in descs:
        v, f = I.batch_mesh(d)
        meshes.append((v, f))
        dev.append((torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda(), d["k"]))
    x_h = np.concatenate([I.complex_vector(3 * f.shape[0], d["seed"]) for d, (_, f) in zip(descs, meshes)])
    M = x_h.shape[0]
    stream = torch.cuda.current_stream()

    def measure(prm, label):
        cdt = torch.complex128 if prm.precision == hmx.FP64 else torch.complex64
        xd = torch.from_numpy(x_h).to(cdt).cuda()

        def step():
            op = hmx.build_batch(dev, bary, w, kern=hmx.HELMHOLTZ, prm=prm, stream=stream)
            return op, op.matvec(xd, stream=stream)

        ms, aca = timed_steps(step, args.steps, args.warmup)
        op, y = step()
        torch.cuda.synchronize()
        info = op.info
        mv = product_ms(op, xd, y, stream, args.matvec_reps)
        y_h = y.cpu().numpy().astype(np.complex128)
        err = worst = None
        if oracle is not None:  # the oracle leg: sampled rows of every mesh
            err, worst = batch_errors(oracle, meshes, descs, bary, w, x_h, y_h, op.mesh_offsets())
            log(f"{label}: errors {err:.3e} (worst mesh {worst:.3e})")
        log(f"{label}: {ms:.1f} ms/step, product {mv:.3f} ms")
        res = {"ms_per_step": round(ms, 3), "h_build_s": round(info["t_total_ms"] / 1e3, 4),
               "h_matvec_ms": round(mv, 4), "rel_err": err, "rel_err_worst_mesh": worst,
               "build_phases_ms": {k2: round(info[k2], 2) for k2 in
                                   ("t_tree_ms", "t_blocks_ms", "t_near_ms", "t_aca_ms")},
               "sizes": sizes(info), "pool_used_bytes": info["factor_bytes"],
               "fallback_rate": info["overflow_blocks"] / max(info["n_far"], 1),
               "aca_rounds": info["aca_rounds"], "predicted_entries": info["predicted_entries"]}
        return res, info, aca, mv, op

    nm = int(args.near_mode == "otf")  # the same near-field policy in both forms
    plain_prm = hmx.params(tol=1e-3, leaf_size=64, eta=1.5, precision=hmx.FP64, near_mode=nm)
    plain, _, _, _, op = measure(plain_prm, "plain FP64 batch")
    op.close()
    model.install()
    try:
        base = hmx.params(tol=1e-3, leaf_size=64, eta=1.5, precision=hmx.FP32_MIXED,
                          rank_model=hmx.RANK_LEARNED, near_mode=nm)
        t0 = time.perf_counter()
        tuned, tune_ms = hmx.autotune_batch(dev, bary, w, kern=hmx.HELMHOLTZ, prm=base,
                                            cache_path=args.tune_cache, stream=stream)
        tune_s = time.perf_counter() - t0
        sched = {k2: getattr(tuned, k2) for k2 in ("max_far_mn", "aca_big_mn", "aca_gram_min_mn",
                                                   "aca_mid_threads", "aca_big_threads",
                                                   "aca_small_mn", "aca_wave", "aca_serial")}
        log(f"autotuned batch schedule in {tune_s:.1f} s: {sched} ({tune_ms:.1f} ms)")
        tgt, info, aca, mv, op = measure(tuned, "FP32 + learned + autotuned batch")
        # the same schedule without the learned layout: the product must be bit-identical
        adapt_prm = hmx.params(**{**{k2: getattr(tuned, k2) for k2, _ in hmx.Params._fields_},
                                  "rank_model": hmx.RANK_ADAPTIVE, "struct_size": tuned.struct_size})
        op_a = hmx.build_batch(dev, bary, w, kern=hmx.HELMHOLTZ, prm=adapt_prm, stream=stream)
        xd = torch.from_numpy(x_h).to(torch.complex64).cuda()
        same = bool(torch.equal(op.matvec(xd), op_a.matvec(xd)))
        adapt_bytes = op_a.info["bytes"]
        op_a.close()
    finally:
        hmx.set_rank_model(None)
    tgt.update({"schedule": sched, "autotune_s": round(tune_s, 1),
                "product_equals_adaptive_same_schedule": same,
                "adaptive_same_schedule_bytes": adapt_bytes})
    extra = {
        "h_build_s": tgt["h_build_s"],
        "h_matvec_ms": tgt["h_matvec_ms"],
        "rel_err": tgt["rel_err"],
        "rel_err_worst_mesh": tgt["rel_err_worst_mesh"],
        "kernel_evals_per_s": info["kernel_evals"] / (info["t_total_ms"] / 1e3),
        "target": tgt,
        "plain_fp64": plain,
        "speedup_vs_plain_fp64": round(plain["ms_per_step"] / tgt["ms_per_step"], 3),
        "rank_model": {"training_blocks": int(sum(len(r) for r in ranks)),
                       "epochs": args.train_epochs, "train_s": round(train_s, 2),
                       "alpha": model.alpha, "beta": model.beta,
                       "final_loss": float(model.history[-1])},
    }
    extra.update(rooflines(info, aca, mv, M, 8, "fp32", near_stored=nm == 0))
    extra["roofline"]["traffic"] = None  # counters were taken on the sphere workload
    op.close()
    cpu = None
    if oracle is not None:
        # bounded sample: the oracle's plain FP64 H-build + product of the first 8 meshes,
        # scaled by points
        c0 = time.perf_counter()
        m_sample = 0
        for (v, f), d in list(zip(meshes, descs))[:8]:
            P, Wq = oracle.quad_points(v, f, bary, w)
            Ho = oracle.HMatrix(P, Wq, oracle.HELMHOLTZ, d["k"], leaf=64, eta=1.5, tol=1e-3)
            Ho.matvec(I.complex_vector(P.shape[0], d["seed"]))
            Ho.close()
            m_sample += P.shape[0]
        c1 = time.perf_counter()
        cpu = {"value": round((c1 - c0) * 1e3 * M / m_sample, 1),
               "unit": "ms per step (H-build + one H-matvec), scaled by points",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"first 8 of the 64 meshes ({m_sample} of {M} points) in {c1 - c0:.2f} s, "
                         "plain FP64, scaled linearly by points"}
    extra["cpu_baseline"] = cpu
    config = {"workload": f"64 seeded ellipsoids ({M} points), Helmholtz k U[2,30], leaf 64, "
                          "eta 1.5, ACA tol 1e-3: FP32 mixed + learned rank layout (network "
                          "trained on the L6 sphere's FP64 and FP32 ranks) + autotuned batch "
                          "schedule, against the plain FP64 batch"
                          + (" (both with the near field computed in the product)" if nm else "")}
    line(args, tgt["ms_per_step"], "fp32", config, extra)


def run_radiation(args, torch, oracle, hmx, I):
    """The L6 sphere's quadrature (245 760 sources, k = 40) radiating onto a 512 x 512 grid in
    the plane z = 0.2 through the sphere: the operator between different point sets."""
    v, f = I.icosphere(args.level)
    bary, w = I.rule_3pt()
    prec = hmx.FP64 if args.precision == "fp64" else hmx.FP32_MIXED
    cdt = torch.complex128 if prec == hmx.FP64 else torch.complex64
    prm = hmx.params(tol=1e-3, leaf_size=64, eta=1.5, precision=prec)
    stream = torch.cuda.current_stream()
    vd, fd = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    xyzw = hmx.quad_points(vd, fd, bary, w, stream=stream)
    nside = 512
    g = np.linspace(-2.0, 2.0, nside)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    T = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 0.2)], 1)
    td = torch.from_numpy(np.ascontiguousarray(T.T)).cuda()
    Mt, Ms = T.shape[0], xyzw.shape[1]
    x_h = I.complex_vector(Ms, 0)
    xd = torch.from_numpy(x_h).to(cdt).cuda()
    torch.cuda.synchronize()
    log(f"bench radiation: {Ms} sources -> {Mt} grid targets, k={args.k}, precision={args.precision}")

    def step():
        op = hmx.build_rect(td, xyzw, kern=hmx.HELMHOLTZ, k=args.k, prm=prm, stream=stream)
        return op, op.matvec(xd, stream=stream)

    ms_step, aca = timed_steps(step, args.steps, args.warmup)
    op, y = step()
    torch.cuda.synchronize()
    info = op.info
    mv_ms = product_ms(op, xd, y, stream, args.matvec_reps)
    log(f"matvec {mv_ms:.3f} ms (median of {args.matvec_reps})")
    y_h = y.cpu().numpy().astype(np.complex128)
    cpu, rel_err = None, None
    if args.cpu_baseline == "on":
        # the oracle leg: dense rows at sampled targets, timed, and the GPU product's error there
        P, Wq = oracle.quad_points(v, f, bary, w)
        rows = np.sort(np.random.default_rng(99).choice(Mt, args.sample_rows, replace=False))
        c0 = time.perf_counter()
        yr = oracle.rect_matvec(T, P, Wq, oracle.HELMHOLTZ, args.k, x_h, rows=rows)
        c1 = time.perf_counter()
        rel_err = float(np.linalg.norm(y_h[rows] - yr) / np.linalg.norm(yr))
        log(f"rel_err on {args.sample_rows} sampled targets: {rel_err:.3e}")
        cpu = {"value": round((c1 - c0) * 1e3 * Mt / len(rows), 1),
               "unit": "ms per dense product at all targets (oracle, no H-matrix)",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"{len(rows)} dense target rows in {c1 - c0:.2f} s, scaled to the "
                         f"{Mt} targets (the oracle has no H-matrix between point sets)"}
    build_s = info["t_total_ms"] / 1e3
    extra = {
        "h_build_s": round(build_s, 4),
        "h_matvec_ms": round(mv_ms, 4),
        "rel_err": rel_err,
        "kernel_evals_per_s": info["kernel_evals"] / build_s if build_s > 0 else None,
        "build_phases_ms": {k2: round(info[k2], 2) for k2 in
                            ("t_tree_ms", "t_blocks_ms", "t_near_ms", "t_aca_ms")},
        "sizes": sizes(info),
        "shape": [Mt, Ms],
    }
    extra.update(rooflines(info, aca, mv_ms, Mt + Ms, 16 if prec == hmx.FP64 else 8, args.precision))
    extra["roofline"]["traffic"] = None  # counters were taken on the sphere workload
    extra["cpu_baseline"] = cpu
    op.close()
    config = {"workload": f"unit icosphere L{args.level} quadrature ({Ms} sources) radiating onto a "
                          f"{nside} x {nside} grid (z = 0.2, [-2, 2]^2, {Mt} targets), Helmholtz "
                          f"k={args.k:g}, leaf 64, eta 1.5, ACA tol 1e-3, {args.precision}"}
    line(args, ms_step, args.precision, config, extra)


# ALU ceiling of the dense on-the-fly product (evaluations per second), from the VALU
# instructions the built kernel issues per evaluation of the Helmholtz kernel (SQ_INSTS_VALU and
# SQ_INSTS_VALU_TRANS_* over the 61 440-point product): FP64 mode 100.8, one of them
# transcendental (the reciprocal square root); FP32 mode 42.4, three transcendental.  A wave64
# VALU instruction occupies a 16-lane SIMD for 4 cycles; the transcendentals overlap with the
# rest (the measured FP32 rate is above what a serial 16-cycle transcendental would allow), so
# 4 x 99.8 = 399 and 4 x 39.4 = 158 SIMD cycles per 64 evaluations, over 1024 SIMDs at 2.4 GHz.
DENSE_ALU_CYCLES = {"fp64": 4 * (100.8 - 1.0), "fp32": 4 * (42.4 - 3.0)}
DENSE_ALU_PEAK = {p: 1024 * 2.4e9 * 64 / c for p, c in DENSE_ALU_CYCLES.items()}


def run_dense(args, torch, oracle, hmx, I):
    """The dense operator on the fly (tol <= 0): L3 sphere, 3 840 points, k = 5, and the same
    kernel at L5 (61 440 points), where it fills the GPU."""
    bary, w = I.rule_3pt()
    prec = hmx.FP64 if args.precision == "fp64" else hmx.FP32_MIXED
    cdt = torch.complex128 if prec == hmx.FP64 else torch.complex64
    stream = torch.cuda.current_stream()
    k = 5.0
    rates = {}
    for level in (3, 5):
        v, f = I.icosphere(level)
        vd, fd = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
        M = 3 * f.shape[0]
        x_h = I.complex_vector(M, 0)
        xd = torch.from_numpy(x_h).to(cdt).cuda()
        prm = hmx.params(tol=0.0, precision=prec)

        def step():
            op = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=k, prm=prm, stream=stream)
            return op, op.matvec(xd, stream=stream)

        if level == 3:
            ms_step, _ = timed_steps(step, args.steps, args.warmup)
        op, y = step()
        torch.cuda.synchronize()
        mv_ms = product_ms(op, xd, y, stream, max(args.matvec_reps, 20))
        rates[level] = (M, mv_ms, M * (M - 1) / (mv_ms * 1e-3))
        log(f"dense L{level}: M={M}, product {mv_ms:.4f} ms, {rates[level][2]:.3e} evaluations/s")
        if level == 3:
            y3, x3, v3, f3 = y.cpu().numpy().astype(np.complex128), x_h, v, f
        op.close()
    cpu, rel_err = None, None
    if args.cpu_baseline == "on":
        # the oracle leg: the full dense product at 3 840 points on all host cores and on one
        P, Wq = oracle.quad_points(v3, f3, bary, w)
        cores = oracle.max_threads()
        c0 = time.perf_counter()
        yr = oracle.dense_matvec(P, Wq, oracle.HELMHOLTZ, k, x3)
        c1 = time.perf_counter()
        oracle.dense_matvec(P, Wq, oracle.HELMHOLTZ, k, x3, nthreads=1)
        c2 = time.perf_counter()
        oracle.dense_matvec(P[:1], Wq[:1], oracle.HELMHOLTZ, k, x3[:1], nthreads=cores)  # restore
        rel_err = float(np.linalg.norm(y3 - yr) / np.linalg.norm(yr))
        cpu = {"value": round((c1 - c0) * 1e3, 3), "unit": "ms per dense product (3 840 points)",
               "cores": cores, "kind": "oracle",
               "sample": f"the full product once; on one core {(c2 - c1) * 1e3:.1f} ms"}
    M3, mv3, r3 = rates[3]
    M5, mv5, r5 = rates[5]
    peak = DENSE_ALU_PEAK[args.precision]
    extra = {
        "dense_matvec_ms": round(mv3, 4),
        "rel_err": rel_err,
        "kernel_evals_per_s": r3,
        "kernel_evals_per_s_61440_points": r5,
        "dense_matvec_ms_61440_points": round(mv5, 4),
        "roofline": {"bound": "alu", "kernel": "hmx::dense_otf_kernel (one evaluation per pair "
                     "and multiply-accumulate, on the fly)", "achieved": round(r5, 1),
                     "peak": round(peak, 1), "unit": "evaluations/s", "frac": round(r5 / peak, 4),
                     "traffic": None, "at": "61 440 points (3 840 points: %.3e/s)" % r3},
        "cpu_baseline": cpu,
    }
    config = {"workload": f"unit icosphere L3 (1280 triangles, {M3} points), Helmholtz k=5, dense "
                          f"operator on the fly, {args.precision}"}
    line(args, ms_step, args.precision, config, extra,
         unit="ms per step (dense operator from device mesh + one product)")


def mie_scattered(T, k, d, nmax=80):
    """Sound-soft unit sphere, incident e^{ik x.d}: the closed-form exterior scattered field."""
    from scipy import special
    r = np.linalg.norm(T, axis=1)
    ct = T @ d / r
    s = np.zeros(len(r), np.complex128)
    for n in range(nmax):
        jn = special.spherical_jn(n, k)
        hn = jn + 1j * special.spherical_yn(n, k)
        hr = special.spherical_jn(n, k * r) + 1j * special.spherical_yn(n, k * r)
        s -= (1j ** n) * (2 * n + 1) * jn / hn * hr * special.eval_legendre(n, ct)
    return s


def run_scattering(args, torch, oracle, hmx, I):
    """The paper's acoustic example at the L6 sphere (40 962 vertices, 245 760 points), k = 40:
    corrected Galerkin P1 single layer, GMRES to 1e-6, scattered field checked against the
    closed-form series at exterior points."""
    v, f = I.icosphere(args.level)
    bary, w = I.rule_3pt()
    d = np.array([0.0, 0.0, 1.0])
    prm = hmx.params(tol=1e-3, leaf_size=64, eta=1.5, regularize=1)
    stream = torch.cuda.current_stream()
    vd, fd = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    xyzw = hmx.quad_points(vd, fd, bary, w, stream=stream)
    pinc = torch.exp(1j * args.k * xyzw[:3].T.to(torch.complex128) @ torch.from_numpy(d).to(torch.complex128).cuda())
    torch.cuda.synchronize()
    log(f"bench scattering: {v.shape[0]} vertices, {xyzw.shape[1]} points, k={args.k}")
    last = {}

    def step():
        if "p1" in last:  # the previous step's space (its operator is closed by then)
            last.pop("p1").close()
        op = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=args.k, prm=prm, stream=stream)
        p1 = hmx.P1(op, vd, fd, bary, w, stream=stream)
        b = p1.project(-pinc, stream=stream)
        lam, it, res = p1.gmres(b, tol=1e-6, restart=200, max_iter=3000, stream=stream)
        last.update(p1=p1, it=it, res=res)
        return op, lam

    ms_step, aca = timed_steps(step, args.steps, args.warmup)
    op, lam = step()
    torch.cuda.synchronize()
    it, res, p1 = last["it"], last["res"], last["p1"]
    info = op.info
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.matvec_reps):
        p1.matvec(lam, stream=stream)
    e1.record(stream)
    e1.synchronize()
    gmv_ms = e0.elapsed_time(e1) / args.matvec_reps
    # scattered field at exterior points against the closed form (outside the timed region)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((400, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    T = u * rng.uniform(1.5, 3.0, 400)[:, None]
    rad = hmx.build_rect(torch.from_numpy(np.ascontiguousarray(T.T)).cuda(), xyzw, kern=hmx.HELMHOLTZ,
                         k=args.k, prm=hmx.params(tol=1e-6))
    ps = rad.matvec(p1.interp(lam)).cpu().numpy()
    ex = mie_scattered(T, args.k, d)
    field_err = float(np.abs(ps - ex).max() / np.abs(ex).max())
    log(f"GMRES {it} iterations, relres {res:.2e}; Galerkin product {gmv_ms:.3f} ms; "
        f"scattered field vs closed form {field_err:.3e}")
    rad.close()
    cpu = None
    if args.cpu_baseline == "on":
        # bounded sample: the oracle's corrected H-build and one product, the solve scaled by the
        # GPU's iteration count (the oracle has no iterative solver)
        P, Wq = oracle.quad_points(v, f, bary, w)
        c0 = time.perf_counter()
        Ho = oracle.HMatrix(P, Wq, oracle.HELMHOLTZ, args.k, leaf=64, eta=1.5, tol=1e-3,
                            mesh=(v, f, bary))
        c1 = time.perf_counter()
        Ho.matvec(I.complex_vector(P.shape[0], 0))
        c2 = time.perf_counter()
        Ho.close()
        cpu = {"value": round(((c1 - c0) + it * (c2 - c1)) * 1e3, 1),
               "unit": "ms per step (corrected H-build + GMRES products), estimated",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"oracle H-build {c1 - c0:.2f} s and one point-operator product "
                         f"{c2 - c1:.2f} s, the solve scaled by {it} iterations"}
    build_s = info["t_total_ms"] / 1e3
    extra = {
        "h_build_s": round(build_s, 4),
        "gmres_iterations": it,
        "gmres_relres": res,
        "galerkin_matvec_ms": round(gmv_ms, 4),
        "scattered_field_rel_err": field_err,
        "build_phases_ms": {k2: round(info[k2], 2) for k2 in
                            ("t_tree_ms", "t_blocks_ms", "t_near_ms", "t_aca_ms")},
        "sizes": sizes(info),
    }
    extra.update(rooflines(info, aca, gmv_ms, xyzw.shape[1], 16, "fp64"))
    extra["cpu_baseline"] = cpu
    p1.close()
    op.close()
    config = {"workload": f"sound-soft unit sphere, icosphere L{args.level} ({v.shape[0]} vertices, "
                          f"{xyzw.shape[1]} points), Helmholtz k={args.k:g}, corrected Galerkin P1 "
                          f"single layer, ACA tol 1e-3, GMRES(200) to 1e-6, fp64"}
    line(args, ms_step, "fp64", config, extra,
         unit="ms per step (corrected H-build from device mesh + GMRES solve of the Galerkin system)")


def mie_pec_far_field(k, th, ph):
    """Far field F (E_s ~ F e^{ikR} / R) of the PEC unit sphere under E_inc = x e^{ikz}: the Mie
    series with a_n = psi_n' / xi_n', b_n = psi_n / xi_n."""
    from scipy import special
    nmax = int(k + 4 * k ** (1 / 3) + 10)
    mu = np.cos(th)
    S1 = np.zeros_like(mu, complex)
    S2 = np.zeros_like(mu, complex)
    pi_prev, pi_cur = np.zeros_like(mu), np.ones_like(mu)
    for n in range(1, nmax + 1):
        jn, djn = special.spherical_jn(n, k), special.spherical_jn(n, k, derivative=True)
        hn = jn + 1j * special.spherical_yn(n, k)
        dhn = djn + 1j * special.spherical_yn(n, k, derivative=True)
        a, b = (jn + k * djn) / (hn + k * dhn), jn / hn
        tau = n * mu * pi_cur - (n + 1) * pi_prev
        c = (2 * n + 1) / (n * (n + 1))
        S1 += c * (a * pi_cur + b * tau)
        S2 += c * (a * tau + b * pi_cur)
        pi_prev, pi_cur = pi_cur, ((2 * n + 1) * mu * pi_cur - (n + 1) * pi_prev) / n
    e_th = np.stack([np.cos(th) * np.cos(ph), np.cos(th) * np.sin(ph), -np.sin(th)], 1)
    e_ph = np.stack([-np.sin(ph), np.cos(ph), np.zeros_like(ph)], 1)
    return ((np.cos(ph) * S2)[:, None] * e_th - (np.sin(ph) * S1)[:, None] * e_ph) / (-1j * k)


class _EmOps:
    """The operators and RWG space of one electromagnetic step, closed together."""

    def __init__(self, single, grads, space):
        self.single, self.grads, self.space = single, grads, space
        self.info = single.info

    def close(self):
        self.space.close()
        for o in [self.single] + self.grads:
            o.close()


def run_em(args, torch, oracle, hmx, I):
    """The paper's electromagnetic example (Section 5.5) on the PEC unit sphere: CFIE with
    beta = 0.5 on RWG elements (corrected single layer and the three gradient kernels as
    H-matrices), GMRES to 1e-6, far field checked against the Mie series."""
    level, k, beta = args.level, args.k, 0.5
    fp32 = args.precision == "fp32"
    prec = hmx.FP32_MIXED if fp32 else hmx.FP64
    cdt = torch.complex64 if fp32 else torch.complex128
    gtol = 1e-5 if fp32 else 1e-6  # c64 vectors: the true residual stalls near 1e-6
    v, f = I.icosphere(level)
    bary, w = I.rule_3pt()
    d, pol = np.array([0.0, 0.0, 1.0]), np.array([1.0, 0.0, 0.0])
    stream = torch.cuda.current_stream()
    vd, fd = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    xyzw = hmx.quad_points(vd, fd, bary, w, stream=stream)
    P = xyzw[:3].T.contiguous()
    ph = torch.exp(1j * k * (P.to(torch.complex128) @ torch.from_numpy(d).to(torch.complex128).cuda()))
    e_inc = (torch.from_numpy(pol).to(torch.complex128).cuda()[:, None] * ph[None, :]).to(cdt).contiguous()
    h_inc = (torch.from_numpy(np.cross(d, pol)).to(torch.complex128).cuda()[:, None] * ph[None, :]).to(cdt).contiguous()
    torch.cuda.synchronize()
    log(f"bench em: {f.shape[0]} triangles, {xyzw.shape[1]} points, {3 * f.shape[0] // 2} edges, k={k}")
    last = {}

    def build_ops():
        single = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=k, stream=stream,
                           prm=hmx.params(tol=1e-3, regularize=1, precision=prec))
        grads = [hmx.build(vd, fd, bary, w, kern=hmx.GRADY_X + i, k=k, stream=stream,
                           prm=hmx.params(tol=1e-3, precision=prec)) for i in range(3)]
        return single, grads

    def step():
        single, grads = build_ops()
        sp = hmx.RWG(single, grads, vd, fd, bary, w, stream=stream)
        b = sp.rhs(beta, e_inc, h_inc, stream=stream)
        x, it, res = sp.gmres(beta, b, tol=gtol, restart=200, max_iter=3000, stream=stream)
        last.update(it=it, res=res, x=x)
        return _EmOps(single, grads, sp), x

    ms_step, aca = timed_steps(step, args.steps, args.warmup)
    ops, x = step()
    torch.cuda.synchronize()
    it, res, sp = last["it"], last["res"], ops.space
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.matvec_reps):
        sp.matvec(beta, x, stream=stream)
    e1.record(stream)
    e1.synchronize()
    cfie_ms = e0.elapsed_time(e1) / args.matvec_reps
    # far field of the current against the Mie series (outside the timed region)
    J = sp.interp(x)[:3].T.cpu().numpy().astype(np.complex128)
    Pn, Wn = P.cpu().numpy(), xyzw[3].cpu().numpy()
    rng = np.random.default_rng(0)
    th, phi = np.arccos(rng.uniform(-1, 1, 100)), rng.uniform(0, 2 * np.pi, 100)
    u = np.stack([np.sin(th) * np.cos(phi), np.sin(th) * np.sin(phi), np.cos(th)], 1)
    Jh = (np.exp(-1j * k * (u @ Pn.T)) * Wn[None, :]) @ J
    F = 1j * k / (4 * np.pi) * (Jh - u * (u * Jh).sum(1, keepdims=True))
    ex = mie_pec_far_field(k, th, phi)
    far_err = float(np.abs(F - ex).max() / np.abs(ex).max())
    log(f"GMRES {it} iterations, relres {res:.2e}; CFIE product {cfie_ms:.3f} ms; "
        f"far field vs Mie series {far_err:.3e}")
    M = xyzw.shape[1]

    def product_bytes(op, nr):
        """Entries read once for nr vectors; per vector x read, xp written and read, y written
        and the permutation twice."""
        i = op.info
        es = 8 if fp32 else 16
        return es * (i["near_entries"] + i["far_entries"] + i["dense_far_entries"]) + nr * (es * 4 * M + 8 * M)

    # the single layer on 4 vectors and each gradient operator on 2, in one product each
    cfie_bytes = product_bytes(ops.single, 4) + sum(product_bytes(g, 2) for g in ops.grads)
    cpu = None
    if args.cpu_baseline == "on":
        # bounded sample: the oracle's four H-builds and one product of each, the solve scaled
        # by the GPU's iteration count (4 single-layer and 6 gradient products per CFIE product)
        Po, Wq = oracle.quad_points(v, f, bary, w)
        xo = I.complex_vector(M, 0)
        c0 = time.perf_counter()
        Hs = oracle.HMatrix(Po, Wq, oracle.HELMHOLTZ, k, leaf=64, eta=1.5, tol=1e-3, mesh=(v, f, bary))
        c1 = time.perf_counter()
        Hs.matvec(xo)
        c2 = time.perf_counter()
        Hs.close()
        Hg = oracle.HMatrix(Po, Wq, oracle.GRADY_X, k, leaf=64, eta=1.5, tol=1e-3)
        c3 = time.perf_counter()
        Hg.matvec(xo)
        c4 = time.perf_counter()
        Hg.close()
        per_it = 4 * (c2 - c1) + 6 * (c4 - c3)
        cpu = {"value": round(((c1 - c0) + 3 * (c3 - c2) + it * per_it) * 1e3, 1),
               "unit": "ms per step (four H-builds + GMRES products), estimated",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"oracle corrected single-layer H-build {c1 - c0:.2f} s and product "
                         f"{c2 - c1:.2f} s, one gradient-kernel H-build {c3 - c2:.2f} s (x3) and "
                         f"product {c4 - c3:.2f} s, the solve scaled by {it} iterations"}
    info = ops.info
    extra = {
        "h_build_s_single_layer": round(info["t_total_ms"] / 1e3, 4),
        "h_build_s_gradients": [round(g.info["t_total_ms"] / 1e3, 4) for g in ops.grads],
        "gmres_iterations": it,
        "gmres_relres": res,
        "cfie_matvec_ms": round(cfie_ms, 4),
        "far_field_rel_err": far_err,
        "sizes": sizes(info),
    }
    extra.update(rooflines(info, aca, cfie_ms, M, 8 if fp32 else 16, args.precision))
    extra["roofline"]["traffic"] = None  # counters were taken on the sphere workload
    extra["roofline_matvec"] = {"bound": "hbm", "achieved": round(cfie_bytes / (cfie_ms * 1e-3) / 1e9, 1),
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": round(cfie_bytes / (cfie_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                "bytes_per_product": cfie_bytes}
    extra["cpu_baseline"] = cpu
    ops.close()
    config = {"workload": f"PEC unit sphere, icosphere L{level} ({f.shape[0]} triangles, {M} points, "
                          f"{3 * f.shape[0] // 2} RWG unknowns), k={k:g}, CFIE beta 0.5 (corrected "
                          f"single layer + 3 gradient kernels), ACA tol 1e-3, GMRES(200) to {gtol:g}, "
                          f"{args.precision}"}
    line(args, ms_step, args.precision, config, extra,
         unit="ms per step (4 H-builds from device mesh + GMRES solve of the CFIE system)")


def run_large(args, torch, oracle, hmx, I):
    """The prolate workload.  --large-shares one: row share 0 of 8 (one GPU's part of the
    row-sharded operator), 100 products replayed in a HIP graph, and the learned layout (a
    network trained on the adaptive ranks of share 1, so share 0 is held out) against plain
    adaptive ACA.  --large-shares all: the whole operator on the one GPU, as its 8 row shares
    built and applied one after the other (each closed before the next), their products summed;
    a step is the 8 builds and products."""
    from paper_1804_00995_amd import rank_model as R
    v, f = I.icosphere(8)
    v = I.ellipsoid(v, (2.0, 1.0, 1.0))
    bary, w = I.rule_3pt()
    M = 3 * f.shape[0]
    k = 120.0
    shares = 8
    whole = args.large_shares == "all"

    # far blocks bounded to 32 768 points (the fastest bound of a sweep at this size)
    def prm(share, **kw):
        return hmx.params(tol=1e-4, leaf_size=128, precision=hmx.FP32_MIXED, row_shares=shares,
                          row_share=share, max_far_mn=32768, **kw)

    vd, fd = torch.from_numpy(v).cuda(), torch.from_numpy(f).cuda()
    x_h = I.complex_vector(M, 0)
    xd = torch.from_numpy(x_h).to(torch.complex64).cuda()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    log(f"bench large: M={M}, " + ("all 8 row shares in turn" if whole else "row share 0 of 8"))

    def graph_ms(op, y, reps):
        g = op.graph(xd, y)
        g.launch(1, stream=stream)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        g.launch(reps, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        g.close()
        return ev0.elapsed_time(ev1) / reps

    if whole:
        def step():
            y = torch.zeros_like(xd)
            infos = []
            for r in range(shares):
                op = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=k, prm=prm(r), stream=stream)
                y += op.matvec(xd, stream=stream)
                infos.append(op.info)
                op.close()
            return _Whole(infos), y

        ms_step, aca = timed_steps(step, args.steps, args.warmup)
        # product of the whole operator: each share's product replayed in a graph, summed
        y = torch.zeros_like(xd)
        mv_ms, build_ms, infos = 0.0, 0.0, []
        for r in range(shares):
            op = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=k, prm=prm(r), stream=stream)
            ys = torch.zeros_like(xd)
            mv_ms += graph_ms(op, ys, args.large_reps)
            y += ys
            infos.append(op.info)
            build_ms += op.info["t_total_ms"]
            op.close()
        torch.cuda.synchronize()
        log(f"whole operator: build {build_ms:.1f} ms, product {mv_ms:.2f} ms (8 shares, "
            f"{args.large_reps} graph replays each)")
        info = _Whole(infos).info
        rows = np.sort(np.random.default_rng(55).choice(M, args.sample_rows, replace=False))
    else:
        # the network: trained on the adaptive ranks of share 1
        op1 = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=k, prm=prm(1), stream=stream)
        feat, ranks = R.block_data(op1)
        op1.close()
        model = R.train(feat, ranks, epochs=30)

        def step():
            op = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=k, prm=prm(0), stream=stream)
            return op, op.matvec(xd, stream=stream)

        ms_step, aca = timed_steps(step, args.steps, args.warmup)
        op, _ = step()
        torch.cuda.synchronize()
        info = op.info
        y = torch.zeros_like(xd)
        mv_ms = graph_ms(op, y, args.large_reps)
        log(f"{args.large_reps} products in one graph: {mv_ms:.3f} ms each")
        perm = op.export_tree()["perm"]
        rb, re = info["row_begin"], info["row_end"]
        rows = np.sort(np.random.default_rng(55).choice(perm[rb:re], args.sample_rows, replace=False))
        op.close()
        model.install()
        try:
            t0 = time.perf_counter()
            opL = hmx.build(vd, fd, bary, w, kern=hmx.HELMHOLTZ, k=k, stream=stream,
                            prm=prm(0, rank_model=hmx.RANK_LEARNED))
            torch.cuda.synchronize()
            t_learned = time.perf_counter() - t0
        finally:
            hmx.set_rank_model(None)
        yL = opL.matvec(xd, stream=stream)
        torch.cuda.synchronize()
        learned = {"trained_on": "adaptive ranks of row share 1 (share 0 held out)",
                   "build_s": round(t_learned, 3), "factor_bytes": opL.info["factor_bytes"],
                   "bytes": opL.info["bytes"], "pool_reserved_bytes": opL.info["pool_reserved_bytes"],
                   "adaptive_pool_reserved_bytes": info["pool_reserved_bytes"],
                   "predicted_entries": opL.info["predicted_entries"],
                   "overflow_blocks": opL.info["overflow_blocks"], "aca_rounds": opL.info["aca_rounds"],
                   "product_equals_adaptive": bool(torch.equal(yL, y))}
        opL.close()
    y_h = y.cpu().numpy().astype(np.complex128)
    rel_err, c0, c1 = None, 0.0, 0.0
    if args.cpu_baseline == "on":
        # the oracle leg: sampled dense rows, timed, and the GPU product's error on them
        P, Wq = oracle.quad_points(v, f, bary, w)
        c0 = time.perf_counter()
        yr = oracle.dense_rows(P, Wq, oracle.HELMHOLTZ, k, x_h, rows)
        c1 = time.perf_counter()
        rel_err = float(np.linalg.norm(y_h[rows] - yr) / np.linalg.norm(yr))
        log(f"rel_err on {args.sample_rows} sampled rows: {rel_err:.3e}")
    cpu = None
    if args.cpu_baseline == "on":
        n_rows = M if whole else info["row_end"] - info["row_begin"]
        cpu = {"value": round((c1 - c0) * 1e3 * n_rows / len(rows), 1),
               "unit": "ms per dense product of the rows measured (oracle, no H-matrix)",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"{len(rows)} dense rows in {c1 - c0:.2f} s, scaled to {n_rows} rows "
                         "(the oracle's H-build does not fit this size in minutes)"}
    build_s = info["t_total_ms"] / 1e3
    extra = {
        "h_build_s": round(build_s, 4),
        "h_matvec_ms": round(mv_ms, 4),
        "rel_err": rel_err,
        "kernel_evals_per_s": info["kernel_evals"] / build_s if build_s > 0 else None,
        "build_phases_ms": {k2: round(info[k2], 2) for k2 in
                            ("t_tree_ms", "t_blocks_ms", "t_near_ms", "t_aca_ms")},
        "sizes": sizes(info),
    }
    if whole:
        extra["shares"] = [{"rows": [i["row_begin"], i["row_end"]], "build_ms": round(i["t_total_ms"], 1),
                            "bytes": i["bytes"], "far_entries": i["far_entries"]} for i in infos]
    else:
        extra["rows"] = [info["row_begin"], info["row_end"]]
        extra["learned_vs_adaptive"] = learned
    extra.update(rooflines(info, aca, mv_ms, M, 8, "fp32"))
    extra["roofline"]["traffic"] = None  # counters were taken on the sphere workload
    extra["cpu_baseline"] = cpu
    part = ("the whole operator as its 8 row shares built and applied in turn"
            if whole else "row share 0 of 8")
    config = {"workload": f"prolate (2,1,1) L8 ({f.shape[0]} triangles, {M} points), k=120, "
                          f"leaf 128, eta 1.5, far blocks <= 32768 points, ACA tol 1e-4, fp32, {part}, "
                          f"{args.large_reps} products in one HIP graph per operator"}
    line(args, ms_step, "fp32", config, extra)


class _Whole:
    """Totals over the row shares of one operator, shaped like Operator.info for the bench."""

    def __init__(self, infos):
        add = ("near_entries", "far_entries", "dense_far_entries", "kernel_evals", "n_near",
               "n_far", "dense_far", "overflow_blocks", "factor_bytes")
        t = {k: sum(i[k] for i in infos) for k in add}
        t.update({k: sum(i[k] for i in infos) for k in ("t_total_ms", "t_tree_ms", "t_blocks_ms",
                                                        "t_near_ms", "t_aca_ms")})
        t["max_rank"] = max(i["max_rank"] for i in infos)
        t["bytes"] = max(i["bytes"] for i in infos)  # one share held at a time
        t["aca_ms"] = [sum(i["aca_ms"][c] for i in infos) for c in range(4)]
        t["aca_bytes"] = [sum(i["aca_bytes"][c] for i in infos) for c in range(4)]
        t["aca_blocks"] = [sum(i["aca_blocks"][c] for i in infos) for c in range(4)]
        t["aca_rounds"] = max(i["aca_rounds"] for i in infos)
        self.info = t

    def close(self):
        pass


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["sphere", "batch", "target", "large", "radiation",
                                           "scattering", "em", "dense"], default="sphere")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--level", type=int, default=None,
                    help="icosphere level (default 6; 5 for the em workload)")
    ap.add_argument("--k", type=float, default=None,
                    help="wavenumber (default 40; 20 for the em workload)")
    ap.add_argument("--matvec-reps", type=int, default=30)
    ap.add_argument("--sample-rows", type=int, default=384)
    ap.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    ap.add_argument("--cpu-one-core", choices=["on", "off"], default="off",
                    help="sphere workload: also time the oracle on one core (about a minute)")
    ap.add_argument("--near-mode", choices=["stored", "otf"], default="otf",
                    help="sphere, batch and target workloads: near blocks computed in each product "
                         "(near_mode 1, the default: faster per step and no near-field memory) or "
                         "stored in the build")
    ap.add_argument("--multi-vectors", type=int, default=0,
                    help="sphere workload: also time the several-vector product for 2, 4, 8, 16 "
                         "vectors up to this many")
    ap.add_argument("--aca-serial", choices=["on", "off"], default="off",
                    help="sphere workload: run the ACA classes one after the other (schedule knob)")
    ap.add_argument("--regularize", choices=["on", "off"], default="off",
                    help="sphere workload: near field with the singular correction")
    ap.add_argument("--large-shares", choices=["one", "all"], default="one",
                    help="large workload: row share 0 of 8, or the whole operator as its 8 shares")
    ap.add_argument("--large-reps", type=int, default=100,
                    help="large workload: products replayed in one graph per operator")
    ap.add_argument("--train-epochs", type=int, default=60,
                    help="target workload: epochs of the rank network's training")
    ap.add_argument("--tune-cache", default=None,
                    help="target workload: autotuner cache file (default: search afresh)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run the copy kernel used to scale the HBM byte counters")
    args = ap.parse_args()
    em = args.workload == "em"  # four operators: one level coarser at the same resolution per wavelength
    args.level = args.level if args.level is not None else (5 if em else 6)
    args.k = args.k if args.k is not None else (20.0 if em else 40.0)
    if args.gpus != 1:
        log("bench.py measures a single GPU; --gpus above 1 is not supported")
        sys.exit(2)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration)
        return

    import torch

    from paper_1804_00995_amd import hmx
    from paper_1804_00995_amd import inputs as I
    oracle = None
    if args.cpu_baseline == "on":  # only the CPU-baseline leg loads the oracle
        import oracle

    {"sphere": run_sphere, "batch": run_batch, "target": run_target, "large": run_large,
     "radiation": run_radiation,
     "scattering": run_scattering, "em": run_em, "dense": run_dense}[args.workload](
        args, torch, oracle, hmx, I)


if __name__ == "__main__":
    main()
