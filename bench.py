#!/usr/bin/env python3
"""Benchmark of the H^2 matrix-vector product for the Galerkin single-layer
matrix G and double-layer matrix K of the 3-D Laplace equation on one MI355X.

Workload (default): the unit sphere of Section 5 (octahedron, every face split
regularly into s*s triangles, vertices projected to radius 1) with s = 512,
i.e. 2,097,152 triangles and 1,048,578 vertices; leaf size 64, eta = 1,
Chebyshev order 4, near-field quadrature order 6 (Table 1 for this n).
x ~ N(0,1) from seeds 501 (G) and 502 (K).

A step is one G x and one K x (all phases of the H^2 product: gather, forward
transformation, coupling, backward transformation, near field, scatter) with
the operators and vectors resident in HBM.  The plain FP64 method is the timed
value; the mixed form (FP32 bases and coupling matrices, FP32 accumulation,
FP64 near field) is timed beside it and its deviation from FP64 reported.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "H² G/K matvec ms & HBM GB/s at 2M triangles; mixed vs FP64 at rel err ≤1e-5"
HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["kernels.hip", "op.hip", "recompress.hip", "panels.hpp", "device.hpp", "op.hpp"]


def sources_digest():
    """sha256 over the library sources that define the product kernels."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2001_05523_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, config):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic.json), or None when the kernels or the workload changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("sources_sha256") != sources_digest() or rec.get("config") != config:
        return None
    return rec.get("traffic_bytes", {}).get(kernel)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def alg_bytes(info, fsz):
    """Algorithmic bytes of one single-vector product, and of its coupling and
    nearfield launches: every stored entry read once, every vector entry read
    once and written once (y read-modify-write counted twice)."""
    vec = 8 * (info["rows"] + 2 * info["rows"] + info["cols"])  # gather/scatter/x/y
    near = 8 * info["near_entries"] + 8 * (info["cols"] + 2 * info["rows"])
    cpl = fsz * info["coupling_entries"] + fsz * (info["col_coeffs"] + 2 * info["row_coeffs"])
    bases = fsz * (info["row_basis_entries"] + info["col_basis_entries"])
    total = near + cpl + bases + vec
    return dict(total=total, near=near, coupling=cpl, bases=bases)


def time_steps(torch, ops, xs, ys, steps, warmup):
    for _ in range(warmup):
        for op, x, y in zip(ops, xs, ys):
            op.matvec(x, y)
    torch.cuda.synchronize()
    for op in ops:
        op.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        for op, x, y in zip(ops, xs, ys):
            op.matvec(x, y)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = [op.phase_times() for op in ops]
    for op in ops:
        op.set_timing(False)
    return (t1 - t0) * 1e3 / steps, phases


def cpu_baseline(verts, tris, q, rows_g, rows_k, x_g, x_k):
    import oracle
    oracle.build(force=False)
    threads = oracle.get_threads()
    t0 = time.perf_counter()
    yg = oracle.slp_rows(verts, tris, q, rows_g, x_g)
    t1 = time.perf_counter()
    yk = oracle.dlp_rows(verts, tris, q, rows_k, x_k)
    t2 = time.perf_counter()
    return dict(yg=yg, yk=yk, tg=t1 - t0, tk=t2 - t1, threads=threads)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--s", type=int, default=512, help="faces split s x s (n = 8 s^2)")
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--q-near", type=int, default=6)
    ap.add_argument("--tol", type=float, default=1e-6, help="recompression tolerance (0: off)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle rows per operator (0: one per thread)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 2 GiB device copy 5 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the H^2 product is measured on one MI355X "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2001_05523_amd as h2b

    torch.cuda.init()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    verts, tris = synth.octa_sphere(args.s)
    nt, nv = len(tris), len(verts)
    log("mesh s=%d: %d triangles, %d vertices (%.1f s)" % (args.s, nt, nv, time.perf_counter() - t0))
    x_g = synth.random_vector(nt, 501)
    x_k = synth.random_vector(nv, 502)

    mesh = h2b.Mesh(verts, tris)
    common = dict(leaf=args.leaf, order_m=args.order, q_near=args.q_near, mesh=mesh,
                  recompress_tol=args.tol)
    ops, assembly_s = {}, {}
    kinds = [("G", "slp", "f64"), ("K", "dlp", "f64")]
    if not args.no_mixed:
        kinds += [("G32", "slp", "f32"), ("K32", "dlp", "f32")]
    for name, kern, fd in kinds:
        t0 = time.perf_counter()
        ops[name] = h2b.Operator(kernel=kern, farfield_dtype=fd, **common)
        torch.cuda.synchronize()
        assembly_s[name] = time.perf_counter() - t0
        inf = ops[name].info()
        log("assembled %s (%s): %.1f s, near %.2f GB, far %.2f GB, %d far / %d near blocks, "
            "mean rank %.1f / %.1f" % (name, fd, assembly_s[name], inf["bytes_near"] / 1e9,
                                       inf["bytes_far"] / 1e9, inf["nfar"], inf["nnear"],
                                       inf["mean_rank_row"], inf["mean_rank_col"]))

    Xg = torch.tensor(x_g, device=dev)
    Xk = torch.tensor(x_k, device=dev)
    Yg = torch.zeros(nt, dtype=torch.float64, device=dev)
    Yk = torch.zeros(nt, dtype=torch.float64, device=dev)

    # one clean product of each for accuracy
    def single(op, X):
        Y = torch.zeros(nt, dtype=torch.float64, device=dev)
        op.matvec(X, Y)
        torch.cuda.synchronize()
        return Y.cpu().numpy()

    y = {name: single(ops[name], Xg if name.startswith("G") else Xk) for name in ops}

    ms64, ph64 = time_steps(torch, [ops["G"], ops["K"]], [Xg, Xk], [Yg, Yk], args.steps, args.warmup)
    log("FP64 step (G x + K x): %.3f ms" % ms64)
    res = {}
    if not args.no_mixed:
        ms32, ph32 = time_steps(torch, [ops["G32"], ops["K32"]], [Xg, Xk], [Yg, Yk], args.steps,
                                args.warmup)
        log("mixed step: %.3f ms" % ms32)

    # per-operator detail
    detail = {}
    dominant = None
    for name, ph in (("G", ph64[0]), ("K", ph64[1])) + ((("G32", ph32[0]), ("K32", ph32[1]))
                                                         if not args.no_mixed else ()):
        inf = ops[name].info()
        fsz = 4 if name.endswith("32") else 8
        b = alg_bytes(inf, fsz)
        ms = sum(ph.values())
        d = dict(ms=ms, phases_ms=ph, alg_bytes=b["total"], gbps=b["total"] / ms / 1e6,
                 coupling_gbps=b["coupling"] / ph["coupling"] / 1e6,
                 near_gbps=b["near"] / ph["nearfield"] / 1e6,
                 bytes_near=inf["bytes_near"], bytes_far=inf["bytes_far"],
                 nfar=inf["nfar"], nnear=inf["nnear"], assembly_s=assembly_s[name],
                 mean_rank=(inf["mean_rank_row"], inf["mean_rank_col"]),
                 max_rank=(inf["max_rank_row"], inf["max_rank_col"]))
        detail[name] = d
        if not name.endswith("32"):
            for kname, ms_k, by in (("coupling", ph["coupling"], b["coupling"]),
                                    ("nearfield", ph["nearfield"], b["near"])):
                if dominant is None or ms_k > dominant[2]:
                    dominant = (name, kname, ms_k, by)
    for base in ("G", "K"):
        if not args.no_mixed:
            a, r = y[base + "32"], y[base]
            detail[base + "32"]["rel_diff_vs_fp64"] = float(np.linalg.norm(a - r) / np.linalg.norm(r))
    step_bytes = detail["G"]["alg_bytes"] + detail["K"]["alg_bytes"]
    traffic_config = {"s": args.s, "leaf": args.leaf, "order": args.order, "q_near": args.q_near,
                      "tol": args.tol}

    out = {
        "metric": METRIC,
        "value": round(ms64, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms64, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "unit sphere (octahedron split s=%d, %d triangles, %d vertices): one G x "
                        "and one K x per step, H^2 Chebyshev order %d recompressed to %g, leaf %d, "
                        "eta 1, q_near %d" % (args.s, nt, nv, args.order, args.tol, args.leaf, args.q_near),
            "triangles": nt, "vertices": nv, "order_m": args.order, "leaf": args.leaf,
            "q_near": args.q_near, "recompress_tol": args.tol, "x_seeds": [501, 502],
        },
        "step_gbps": round(step_bytes / ms64 / 1e6, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": "%s %s panel product (k_rowpanel<double, double, double, %d, *>)"
                      % (dominant[0], dominant[1], 2 if dominant[1] == "coupling" else 3),
            "achieved": round(dominant[3] / dominant[2] / 1e6, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dominant[3] / dominant[2] / 1e6 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("%s %s" % dominant[:2], traffic_config),
            "alg_bytes": dominant[3],
            "avg_launch_ms": round(dominant[2], 4),
        },
        "detail": detail,
    }
    if not args.no_mixed:
        out["mixed"] = {"ms_per_step": round(ms32, 4), "speedup_vs_fp64": round(ms64 / ms32, 3),
                        "rel_diff_G": detail["G32"]["rel_diff_vs_fp64"],
                        "rel_diff_K": detail["K32"]["rel_diff_vs_fp64"],
                        "step_gbps": round((detail["G32"]["alg_bytes"] + detail["K32"]["alg_bytes"])
                                           / ms32 / 1e6, 1)}

    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 5 copies of %d bytes" % (src.numel() * 8))
        del src, dst

    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        nthreads = oracle.get_threads()
        nrows = args.cpu_rows or nthreads
        rng = np.random.default_rng(503)
        rows_g = np.sort(rng.choice(nt, nrows, replace=False))
        rows_k = np.sort(rng.choice(nt, nrows, replace=False))
        log("oracle: %d G rows and %d K rows on %d threads" % (nrows, nrows, nthreads))
        cb = cpu_baseline(verts, tris, args.q_near, rows_g, rows_k, x_g, x_k)
        est_ms = (cb["tg"] / nrows + cb["tk"] / nrows) * nt * 1e3
        log("oracle rows: G %.1f s, K %.1f s" % (cb["tg"], cb["tk"]))
        out["cpu_baseline"] = {
            "value": est_ms, "unit": "ms", "cores": cb["threads"], "kind": "oracle",
            "sample": "%d rows of G and %d rows of K (seed 503) of the same 2M-triangle operators, "
                      "dense FP64 quadrature, timed %.1f s + %.1f s and scaled by n/rows to one "
                      "dense G x + K x" % (nrows, nrows, cb["tg"], cb["tk"]),
        }
        acc = {}
        for name in ops:
            ref = cb["yg"] if name.startswith("G") else cb["yk"]
            rows = rows_g if name.startswith("G") else rows_k
            got = y[name][rows]
            acc[name] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        out["sampled_row_rel_err"] = acc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
