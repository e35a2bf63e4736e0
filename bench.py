#!/usr/bin/env python3
"""Benchmark of the H^2 matrix-vector product for the Galerkin single-layer
matrix G and double-layer matrix K of the 3-D Laplace equation on one MI355X.

Workload (default): the unit sphere of Section 5 (octahedron, every face split
regularly into s*s triangles, vertices projected to radius 1) with s = 512,
i.e. 2,097,152 triangles and 1,048,578 vertices; leaf size 64, eta = 1,
Chebyshev order 4, near-field quadrature order 6 (Table 1 for this n).
x ~ N(0,1) from seeds 501 (G) and 502 (K).

A step is G x, G^T x, K x and K^T x (every phase of the H^2 product: gather,
forward transformation, coupling, backward transformation, near field,
scatter; the near field runs on its own stream beside the far field) with the
operators and vectors resident in HBM.  The plain FP64 method is the timed
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
KERNEL_SOURCES = ["kernels.hip", "symnear.hip", "symcpl.hip", "op.hip", "transform.hip", "recompress.hip", "panels.hpp",
                  "device.hpp", "op.hpp"]


def code_text(src):
    """The code of a C++/HIP source without its comments and blank lines (the
    HBM traffic of a kernel depends on its code, not on its comments)."""
    import re
    src = re.sub(rb"/\*.*?\*/", b"", src, flags=re.S)
    src = re.sub(rb"//[^\n]*", b"", src)
    return b"\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def sources_digest(read=None):
    """sha256 over the code of the library sources that define the product
    kernels (read(name) -> bytes; default: the files in the tree)."""
    import hashlib
    if read is None:
        def read(f):
            with open(os.path.join(ROOT, "paper_2001_05523_amd", "csrc", f), "rb") as fh:
                return fh.read()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(code_text(read(f)))
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


def alg_bytes(info, fsz, trans=False):
    """Algorithmic bytes of one single-vector product A x (or A^T x), and of its
    coupling and nearfield launches: every stored entry read once, every
    vector entry read once and written once (y read-modify-write counted
    twice)."""
    nin, nout = (info["rows"], info["cols"]) if trans else (info["cols"], info["rows"])
    hin, hout = (info["row_coeffs"], info["col_coeffs"]) if trans else (info["col_coeffs"], info["row_coeffs"])
    vec = 8 * (nout + 2 * nout + nin)  # gather/scatter/x/y
    if info["near_sym_entries"] > 0:
        # once-per-pair storage: entries, column sums written and read back,
        # corrections (value, index, gathered x), their row pointers
        near = (8 * info["near_sym_entries"] + 16 * info["near_sym_columns"]
                + 20 * info["near_sym_corrections"] + 8 * nout + 8 * (nin + 2 * nout))
    else:
        near = 8 * info["near_entries"] + 8 * (nin + 2 * nout)
    if info.get("cpl_sym_entries", 0) > 0:
        # once-per-pair coupling: entries, column sums written and read back
        cpl = fsz * info["cpl_sym_entries"] + 2 * fsz * info["cpl_sym_columns"] + fsz * (hin + 2 * hout)
    else:
        cpl = fsz * info["coupling_entries"] + fsz * (hin + 2 * hout)
    bases = fsz * (info["row_basis_entries"] + info["col_basis_entries"])
    total = near + cpl + bases + vec
    return dict(total=total, near=near, coupling=cpl, bases=bases)


def kernel_name(op, phase, info):
    """Kernels that make up a product phase, for the roofline record."""
    if phase == "coupling":
        if info.get("cpl_sym_entries", 0) > 0:
            return ("%s coupling stored once per pair of clusters, A x and A^T x launches (k_cplsym "
                    "+ k_cplreduce)" % op)
        return "%s coupling, A x and A^T x launches (k_rowpanel<double, double, double, 2, 1, 4>)" % op
    if info["near_sym_entries"] > 0:
        return ("%s nearfield stored once per pair of leaves, A x and A^T x launches (k_nearsym<false|true> "
                "+ k_symreduce)" % op)
    return "%s nearfield, A x and A^T x launches (k_rowpanel<double, double, double, 3, 4, 2>)" % op


def time_steps(torch, items, steps, warmup, streams=None):
    """Times `steps` passes over items = [(op, x, y, trans), ...] after `warmup`
    untimed passes, with the operators' phase events recorded on the streams
    the phases run on.  With `streams` (one torch stream per item, or None)
    the products of different operators are issued on their own streams, so
    that they may run concurrently; products on one operator share a stream
    (they share its work vectors).  Returns ms per pass and each operator's
    mean phase times (over its products in the pass)."""
    ops = []
    for it in items:
        if all(it[0] is not o for o in ops):
            ops.append(it[0])
    streams = streams or [None] * len(items)
    for _ in range(warmup):
        for (op, x, y, tr), s in zip(items, streams):
            op.matvec(x, y, trans=tr, stream=s)
    torch.cuda.synchronize()
    for op in ops:
        op.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        for (op, x, y, tr), s in zip(items, streams):
            op.matvec(x, y, trans=tr, stream=s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = [op.phase_times() for op in ops]
    for op in ops:
        op.set_timing(False)
    return (t1 - t0) * 1e3 / steps, phases


def time_product(torch, op, x, y, trans, reps=10):
    """ms per product of one operator and direction alone (no events)."""
    op.matvec(x, y, trans=trans)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        op.matvec(x, y, trans=trans)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


def cpu_baseline(verts, tris, q, sample, xin):
    """Oracle rows of G and K on the host's cores."""
    import oracle
    oracle.build(force=False)
    threads = oracle.get_threads()
    fn = {"G": (oracle.slp_rows, False), "K": (oracle.dlp_rows, False)}
    y, t = {}, {}
    for p, rows in sample.items():
        f, tr = fn[p]
        t0 = time.perf_counter()
        y[p] = f(verts, tris, q, rows, xin[p], trans=tr)
        t[p] = time.perf_counter() - t0
    return dict(y=y, t=t, threads=threads)


MFMA_F32_PEAK_TFLOPS = 157.3


def batching(torch, h2b, synth, reps):
    """Many right-hand sides and many meshes (FP32 far field, FP64 nearfield):
    64 N(0,1) right-hand sides on the 32,768-triangle sphere (order 4
    recompressed to 1e-6, leaf 32, q_near 4) with the autotuned matrix-core
    coupling, and 16 spheres / ellipsoids of 2,048 to 32,768 triangles (semi-
    axes U[0.5, 2]) captured into one graph."""
    dev = torch.device("cuda:0")
    res = {}
    v, t = synth.octa_sphere(64)
    for name, kern in (("G", "slp"), ("K", "dlp")):
        op = h2b.Operator(v, t, kernel=kern, leaf=32, order_m=4, q_near=4, recompress_tol=1e-6,
                          farfield_dtype="f32")
        ref = h2b.Operator(v, t, kernel=kern, leaf=32, order_m=4, q_near=4, recompress_tol=1e-6)
        inf = op.info()
        tune_us = op.tune(64)
        X = torch.tensor(synth.random_vector(op.shape[1], 601, cols=64), device=dev).t().contiguous().t()
        Y = torch.zeros((op.shape[0], 64), dtype=torch.float64, device=dev).t().contiguous().t()
        op.matvec(X, Y)
        torch.cuda.synchronize()
        # accuracy of two columns against the FP64 single-vector products
        Y.zero_()
        op.matvec(X, Y)
        errs = []
        for c in (0, 63):
            y1 = torch.zeros(op.shape[0], dtype=torch.float64, device=dev)
            ref.matvec(X[:, c].contiguous(), y1)
            errs.append(float(torch.linalg.norm(Y[:, c] - y1) / torch.linalg.norm(y1)))
        op.set_timing(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            op.matvec(X, Y)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        ph = op.phase_times()
        op.set_timing(False)
        flops = 2.0 * inf["coupling_entries"] * 64
        tf = flops / ph["coupling"] / 1e9
        res[name + "_64rhs"] = {
            "ms": round(ms, 4), "rhs_per_s": round(64 / ms * 1e3, 1), "phases_ms": ph,
            "coupling_tflops": round(tf, 2), "coupling_mfma_frac": round(tf / MFMA_F32_PEAK_TFLOPS, 4),
            "coupling_flops": flops, "tune_us": round(tune_us, 2), "rel_err_vs_fp64": errs,
        }
        log("%s x 64 rhs: %.3f ms (coupling %.3f ms, %.1f TFLOP/s on matrix cores)" % (name, ms, ph["coupling"], tf))
        del op, ref
    rng = np.random.default_rng(602)
    ops, items, ntri, abytes = [], [], 0, 0.0
    for k in range(16):
        s = int(rng.integers(16, 65))
        a, b, c = rng.uniform(0.5, 2.0, size=3)
        if k % 2 == 0:
            a = b = c
        vv, tt = synth.ellipsoid(s, a, b, c)
        kern = "slp" if k % 3 else "dlp"
        op = h2b.Operator(vv, tt, kernel=kern, leaf=32, order_m=4, q_near=4, recompress_tol=1e-6,
                          farfield_dtype="f32")
        x = torch.tensor(synth.random_vector(op.shape[1], 610 + k), device=dev)
        y = torch.zeros(op.shape[0], dtype=torch.float64, device=dev)
        ops.append(op)
        items.append((op, x, y))
        ntri += len(tt)
        # the merged batch reads the full nearfield of G (not the once-per-pair form)
        inf = dict(op.info())
        inf["near_sym_entries"] = 0
        inf["cpl_sym_entries"] = 0
        abytes += alg_bytes(inf, 4)["total"]

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    batch = h2b.Batch(items)
    bms = timed(batch.launch, 4 * reps)
    ems = timed(lambda: [op.matvec(x, y) for op, x, y in items], 2 * reps)
    # reference: one product on the largest mesh of the list alone
    big = max(range(16), key=lambda i: ops[i].shape[0])
    bop, bx, by = items[big]
    inf = bop.info()
    sms = timed(lambda: bop.matvec(bx, by), 4 * reps)
    res["batch16"] = {"meshes": 16, "triangles": ntri, "merged": True, "graph_launch_ms": round(bms, 4),
                      "eager_sequence_ms": round(ems, 4), "ns_per_triangle": round(bms * 1e6 / ntri, 3),
                      "alg_bytes": abytes, "gbps": round(abytes / bms / 1e6, 1),
                      "largest_mesh_alone": {"triangles": inf["rows"], "ms": round(sms, 4),
                                             "ns_per_triangle": round(sms * 1e6 / inf["rows"], 3),
                                             "gbps": round(alg_bytes(inf, 4)["total"] / sms / 1e6, 1)}}
    log("batch of 16 meshes (%d triangles): one graph launch %.3f ms (%.2f ns per triangle, %.0f GB/s), "
        "eager sequence %.3f ms; largest mesh alone %.3f ms (%.2f ns per triangle)"
        % (ntri, bms, bms * 1e6 / ntri, abytes / bms / 1e6, ems, sms, sms * 1e6 / inf["rows"]))
    # the same meshes with 64 right-hand sides each
    items64 = []
    for k, (op, _, _) in enumerate(items):
        X = torch.tensor(synth.random_vector(op.shape[1], 630 + k, cols=64), device=dev).t().contiguous().t()
        Y = torch.zeros((64, op.shape[0]), dtype=torch.float64, device=dev).t()
        items64.append((op, X, Y))
    batch64 = h2b.Batch(items64)
    b64 = timed(batch64.launch, 2 * reps)
    e64 = timed(lambda: [op.matvec(X, Y) for op, X, Y in items64], reps)
    res["batch16_64rhs"] = {"meshes": 16, "triangles": ntri, "rhs": 64, "graph_launch_ms": round(b64, 4),
                            "eager_sequence_ms": round(e64, 4),
                            "ns_per_triangle_rhs": round(b64 * 1e6 / ntri / 64, 4)}
    log("batch of 16 meshes x 64 right-hand sides: one graph launch %.3f ms (%.3f ns per triangle and "
        "right-hand side), eager sequence %.3f ms" % (b64, b64 * 1e6 / ntri / 64, e64))
    del batch, batch64
    return res


def neumann_l2_error_u1(verts, tris, t):
    """|| t - <grad u1, n_tau> ||_L2 for u1 = x1^2 - x3^2 on the flat triangles
    (the normal derivative is linear on each triangle, so the three-point
    edge-midpoint rule, exact for quadratics, integrates the square exactly)."""
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    n = cr / (2.0 * area)[:, None]
    err2 = np.zeros(len(tris))
    for p in (0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a)):
        dn = 2.0 * p[:, 0] * n[:, 0] - 2.0 * p[:, 2] * n[:, 2]
        err2 += (t - dn) ** 2 / 3.0
    return float(np.sqrt(np.sum(err2 * area)))


def dtn_solve(torch, h2b, ops, verts, tris, suffixes, ms_gx):
    """Dirichlet-to-Neumann solve G t = (M/2 + K) u for u = u1 = x1^2 - x3^2 on
    the benchmark mesh: right-hand side from the library's mass and K
    products, conjugate gradients to 1e-8 on G (graph-replayed batches of 8
    iterations; once more queued eagerly for comparison)."""
    u = torch.tensor(verts[:, 0] ** 2 - verts[:, 2] ** 2, dtype=torch.float64, device="cuda")
    res = {"problem": "G t = (M/2 + K) u, u = x1^2 - x3^2, CG tol 1e-8 from t = 0, FP64 inner products"}
    sols = {}
    for suffix in suffixes:
        G, K = ops["G" + suffix], ops["K" + suffix]
        b = h2b.dtn_rhs(K, u)
        t = torch.zeros_like(b)
        r = G.cg(b, t, tol=1e-8, max_iter=3000)
        t2 = torch.zeros_like(b)
        re = G.cg(b, t2, tol=1e-8, max_iter=3000, use_graph=False)
        chk = b.clone()
        G.matvec(t, chk, alpha=-1.0)
        torch.cuda.synchronize()
        true_rel = float(torch.linalg.norm(chk) / torch.linalg.norm(b))
        sols[suffix] = t.cpu().numpy()
        it = max(r["iterations"], 1)
        d = {"iterations": r["iterations"], "status": r["status"], "rel_residual": r["rel_residual"],
             "true_rel_residual": true_rel, "solve_ms": round(r["solve_ms"], 2),
             "ms_per_iteration": round(r["solve_ms"] / it, 4),
             "eager_solve_ms": round(re["solve_ms"], 2), "eager_iterations": re["iterations"],
             "l2_error_neumann": neumann_l2_error_u1(verts, tris, sols[suffix])}
        if ms_gx.get(suffix):
            d["iteration_over_product"] = round(r["solve_ms"] / it / ms_gx[suffix], 3)
        if not suffix:
            tp = torch.zeros_like(b)
            rp = G.cg(b, tp, tol=1e-8, max_iter=3000, precond="block_jacobi")
            d["block_jacobi"] = {"iterations": rp["iterations"], "status": rp["status"],
                                 "solve_ms": round(rp["solve_ms"], 2), "rel_residual": rp["rel_residual"],
                                 "rel_diff_vs_cg": float(torch.linalg.norm(tp - t) / torch.linalg.norm(t))}
            log("DtN solve with block-Jacobi: %d iterations, %.1f ms (setup of the inverses included)"
                % (rp["iterations"], rp["solve_ms"]))
        res["f64" if not suffix else "mixed"] = d
        log("DtN solve (%s): %d iterations, %.1f ms (%.3f ms per iteration; eager %.1f ms), "
            "residual %.2e (true %.2e), L2 error %.3e" % ("f64" if not suffix else "mixed", r["iterations"],
                                                         r["solve_ms"], r["solve_ms"] / it, re["solve_ms"],
                                                         r["rel_residual"], true_rel, d["l2_error_neumann"]))
    if "32" in sols:
        res["mixed"]["rel_diff_vs_fp64"] = float(np.linalg.norm(sols["32"] - sols[""]) / np.linalg.norm(sols[""]))
    return res


def ntd_solve(torch, h2b, ops, verts, tris):
    """Neumann-to-Dirichlet solve W u = (M^T/2 - K^T) t on the benchmark mesh,
    W = sum_d C_d^T G C_d from the FP64 G, t the exact normal derivative of
    u1 = x1^2 - x3^2 at the triangle centroids; CG to 1e-8 from u = 0."""
    G, K = ops["G"], ops["K"]
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    cr = np.cross(b - a, c - a)
    n = cr / np.linalg.norm(cr, axis=1)[:, None]
    cen = (a + b + c) / 3.0
    tn = torch.tensor(2.0 * cen[:, 0] * n[:, 0] - 2.0 * cen[:, 2] * n[:, 2], dtype=torch.float64, device="cuda")
    rhs = h2b.ntd_rhs(K, tn)
    x = torch.zeros_like(rhs)
    y = torch.zeros_like(rhs)
    G.hypersingular_matvec(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        G.hypersingular_matvec(rhs, y)
    torch.cuda.synchronize()
    ms_w = (time.perf_counter() - t0) * 1e3 / 5
    r = G.cg(rhs, x, tol=1e-8, max_iter=3000, form="hypersingular")
    u = x.cpu().numpy()
    ex = verts[:, 0] ** 2 - verts[:, 2] ** 2
    # relative nodal error after matching the zero-mean representative
    area = 0.5 * np.linalg.norm(cr, axis=1)
    w1 = np.zeros(len(verts))
    for k in range(3):
        np.add.at(w1, tris[:, k], area / 3.0)
    ex = ex - (w1 @ ex) / w1.sum()
    it = max(r["iterations"], 1)
    d = {"problem": "W u = (M^T/2 - K^T) t, t = d(x1^2 - x3^2)/dn at the centroids, CG tol 1e-8 from u = 0, "
                    "W from the FP64 G",
         "iterations": r["iterations"], "status": r["status"], "rel_residual": r["rel_residual"],
         "solve_ms": round(r["solve_ms"], 2), "ms_per_iteration": round(r["solve_ms"] / it, 4),
         "ms_hypersingular_product": round(ms_w, 4),
         "nodal_rel_err_vs_u1": float(np.max(np.abs(u - ex)) / np.max(np.abs(ex)))}
    log("NtD solve: %d iterations, %.1f ms (%.3f ms per iteration; W x alone %.3f ms), residual %.2e, "
        "nodal error %.3e" % (r["iterations"], r["solve_ms"], r["solve_ms"] / it, ms_w, r["rel_residual"],
                              d["nodal_rel_err_vs_u1"]))
    return d


def hchol_solves(torch, h2b, sizes):
    """The paper's preconditioner (coarsening and H-Cholesky factorisation of
    G to eps_prc, Section 1; eps_prc from the parameter table of Section 5
    for these sizes) on the Dirichlet-to-Neumann system G t = (M/2 + K) u1 of
    smaller spheres: setup stages on the host, the factor's storage, the
    device substitutions per application (HIP events), and CG to 1e-8
    without a preconditioner, with block Jacobi and with the factor."""
    import synth
    res = {}
    for s, eps in sizes:
        v, t = synth.octa_sphere(s)
        G = h2b.Operator(v, t, kernel="slp", leaf=64, order_m=4, q_near=4, recompress_tol=1e-6)
        K = h2b.Operator(kernel="dlp", leaf=64, order_m=4, q_near=4, recompress_tol=1e-6, mesh=G.mesh)
        u = torch.tensor(v[:, 0] ** 2 - v[:, 2] ** 2, dtype=torch.float64, device="cuda")
        b = h2b.dtn_rhs(K, u)
        t0 = time.perf_counter()
        P = h2b.HChol(G, eps)
        build_s = time.perf_counter() - t0
        info = P.info()
        z = torch.zeros_like(b)
        P.apply(b, z)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            P.apply(b, z)
        e1.record()
        torch.cuda.synchronize()
        apply_ms = e0.elapsed_time(e1) / 10
        d = {"triangles": len(t), "eps_prc": eps, "build_s": round(build_s, 2),
             "setup_s": {k: round(info[k], 3) for k in ("convert_s", "coarsen_s", "factor_s", "upload_s")},
             "factor_entries": info["dense_entries"] + info["rk_entries"],
             "factor_bytes_per_row": round(8.0 * (info["dense_entries"] + info["rk_entries"]) / len(t), 1),
             "coarse_entries": info["coarse_entries"], "max_rank": info["max_rank"],
             "substitution_steps": info["steps"], "apply_ms": round(apply_ms, 3),
             "us_per_step": round(1e3 * apply_ms / max(info["steps"], 1), 3)}
        sols = {}
        for name, kw in (("cg", {}), ("block_jacobi", {"precond": "block_jacobi"}),
                         ("hchol", {"precond": "hchol", "hchol": P})):
            x = torch.zeros_like(b)
            r = G.cg(b, x, tol=1e-8, max_iter=3000, **kw)
            sols[name] = x
            d[name] = {"iterations": r["iterations"], "status": r["status"], "solve_ms": round(r["solve_ms"], 2)}
        for name in ("block_jacobi", "hchol"):
            d[name]["rel_diff_vs_cg"] = float(torch.linalg.norm(sols[name] - sols["cg"]) / torch.linalg.norm(sols["cg"]))
        res["sphere_%d" % len(t)] = d
        log("H-Cholesky, %d triangles, eps %.0e: setup %.1f s (%s), factor %.1f MB, apply %.3f ms (%d steps); "
            "CG %d it %.1f ms, block Jacobi %d it %.1f ms, H-Cholesky %d it %.1f ms" % (
                len(t), eps, build_s, ", ".join("%s %.2f" % kv for kv in d["setup_s"].items()),
                8e-6 * d["factor_entries"], apply_ms, info["steps"], d["cg"]["iterations"], d["cg"]["solve_ms"],
                d["block_jacobi"]["iterations"], d["block_jacobi"]["solve_ms"], d["hchol"]["iterations"],
                d["hchol"]["solve_ms"]))
        del P, G, K
        torch.cuda.empty_cache()
    return res


def gca_solve(torch, h2b, mesh, verts, tris, args):
    """Dirichlet-to-Neumann solve with the Green cross approximation (order
    args.gca_order per face direction, tolerance args.gca_tol, bases
    recompressed to args.gca_recompress) for both G and K, no transposed
    copies (the solve uses G x and K x only): setup, storage, product time,
    the error on the stored oracle rows, and the L2 error of the Neumann data
    of u1 = x1^2 - x3^2."""
    res = {"problem": "G t = (M/2 + K) u, u = x1^2 - x3^2, GCA order %d tol %g recompressed to %g, "
                      "block-Jacobi PCG tol 1e-8" % (args.gca_order, args.gca_tol, args.gca_recompress)}
    kw = dict(leaf=args.leaf, order_m=args.gca_order, q_near=args.q_near, gca_tol=args.gca_tol,
              recompress_tol=args.gca_recompress, transposed_copy=False, mesh=mesh)
    gops = {}
    for name, kern in (("G", "slp"), ("K", "dlp")):
        t0 = time.perf_counter()
        gops[name] = h2b.Operator(kernel=kern, **kw)
        torch.cuda.synchronize()
        inf = gops[name].info()
        res[name] = {"setup_s": round(time.perf_counter() - t0, 1), "bytes_far": inf["bytes_far"],
                     "bytes_near": inf["bytes_near"], "mean_rank": (inf["mean_rank_row"], inf["mean_rank_col"]),
                     "max_rank": (inf["max_rank_row"], inf["max_rank_col"])}
        log("GCA %s: setup %.1f s, far %.2f GB, mean ranks %.1f / %.1f" % (
            name, res[name]["setup_s"], inf["bytes_far"] / 1e9, inf["mean_rank_row"], inf["mean_rank_col"]))
    G = gops["G"]
    x = torch.tensor(synth_vector(len(tris)), device="cuda")
    y = torch.zeros_like(x)
    G.matvec(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        G.matvec(x, y)
    torch.cuda.synchronize()
    res["G"]["ms_Ax"] = round((time.perf_counter() - t0) * 1e3 / 5, 4)
    log("GCA G x: %.3f ms" % res["G"]["ms_Ax"])
    # the 1,000 oracle rows stored for this mesh, if present
    gold_path = os.path.join(ROOT, "tests", "golden", "sphere2M_oracle_rows.json")
    if os.path.exists(gold_path) and args.s == 512 and args.q_near == 6 and args.leaf == 64:
        import synth
        with open(gold_path) as fh:
            gold = json.load(fh)
        rows = np.asarray(gold["rows"])
        acc = {}
        for name in ("G", "K"):
            n_in = len(tris) if name == "G" else len(verts)
            xg = torch.tensor(synth.random_vector(n_in, gold[name]["x_seed"]), device="cuda")
            got = (gops[name] @ xg).cpu().numpy()[rows]
            ref = np.asarray(gold[name]["y"])
            acc[name] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        res["oracle_rows_1000"] = acc
        log("GCA on the 1,000 stored oracle rows: G %.3e, K %.3e" % (acc["G"], acc["K"]))
    u = torch.tensor(verts[:, 0] ** 2 - verts[:, 2] ** 2, dtype=torch.float64, device="cuda")
    b = h2b.dtn_rhs(gops["K"], u)
    t = torch.zeros_like(b)
    r = G.cg(b, t, tol=1e-8, max_iter=3000, precond="block_jacobi")
    res["cg"] = {"iterations": r["iterations"], "status": r["status"], "solve_ms": round(r["solve_ms"], 1),
                 "rel_residual": r["rel_residual"]}
    res["l2_error_neumann"] = neumann_l2_error_u1(verts, tris, t.cpu().numpy())
    log("GCA DtN solve: %d iterations, %.1f ms, L2 error %.4e" % (r["iterations"], r["solve_ms"],
                                                                 res["l2_error_neumann"]))
    # Neumann-to-Dirichlet with W from the GCA G and the right-hand side from the GCA K
    a, b3, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    cr = np.cross(b3 - a, c - a)
    n = cr / np.linalg.norm(cr, axis=1)[:, None]
    cen = (a + b3 + c) / 3.0
    tn = torch.tensor(2.0 * cen[:, 0] * n[:, 0] - 2.0 * cen[:, 2] * n[:, 2], dtype=torch.float64, device="cuda")
    rhs = h2b.ntd_rhs(gops["K"], tn)
    uh = torch.zeros_like(rhs)
    r = G.cg(rhs, uh, tol=1e-10, max_iter=3000, form="hypersingular")
    res["ntd"] = {"iterations": r["iterations"], "status": r["status"], "solve_ms": round(r["solve_ms"], 1),
                  "rel_residual": r["rel_residual"],
                  "l2_error_dirichlet": dirichlet_l2_error_u1(verts, tris, uh.cpu().numpy())}
    log("GCA NtD solve: %d iterations, %.1f ms, L2 error of the Dirichlet data %.4e" % (
        r["iterations"], r["solve_ms"], res["ntd"]["l2_error_dirichlet"]))
    return res


def dirichlet_l2_error_u1(verts, tris, uh):
    """|| (u_h - mean) - (u1 - mean) ||_L2 for the P1 function u_h against
    u1 = x1^2 - x3^2 on the flat triangles (collapsed 4 x 4 Gauss rule, exact
    for the quartic integrand; both sides with zero mean, since the Neumann
    data fix u only up to a constant)."""
    z, w = np.polynomial.legendre.leggauss(4)
    t1, w1 = 0.5 * (z + 1.0), 0.5 * w
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    jac = np.linalg.norm(np.cross(b - a, c - b), axis=1)
    num = den = 0.0
    vals, wts = [], []
    for i in range(4):
        for j in range(4):
            u1, u2 = t1[i], t1[i] * t1[j]
            x = a + u1 * (b - a) + u2 * (c - b)
            lam = (1.0 - u1, u1 - u2, u2)
            vh = lam[0] * uh[tris[:, 0]] + lam[1] * uh[tris[:, 1]] + lam[2] * uh[tris[:, 2]]
            vals.append((vh, x[:, 0] ** 2 - x[:, 2] ** 2))
            wts.append(w1[i] * w1[j] * t1[i] * jac)
    tot = sum(wt.sum() for wt in wts)
    mh = sum((wt * vh).sum() for (vh, _), wt in zip(vals, wts)) / tot
    mu = sum((wt * vu).sum() for (_, vu), wt in zip(vals, wts)) / tot
    err2 = sum((wt * ((vh - mh) - (vu - mu)) ** 2).sum() for (vh, vu), wt in zip(vals, wts))
    return float(np.sqrt(err2))


def synth_vector(n):
    import synth
    return synth.random_vector(n, 501)


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
    ap.add_argument("--no-batching", action="store_true", help="skip the many-RHS / many-mesh section")
    ap.add_argument("--no-hchol", action="store_true", help="skip the H-Cholesky preconditioner section")
    ap.add_argument("--no-gca-solve", action="store_true",
                    help="skip the solves with GCA operators (about a minute of setup)")
    ap.add_argument("--gca-order", type=int, default=4)
    ap.add_argument("--gca-tol", type=float, default=1e-6)
    ap.add_argument("--gca-recompress", type=float, default=1e-6,
                    help="recompression tolerance of the GCA bases (0: none)")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the Dirichlet-to-Neumann and Neumann-to-Dirichlet CG solves")
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

    # inputs of the four products: G x, G^T x (x on triangles), K x (x on
    # vertices), K^T x (x on triangles)
    x_gt = synth.random_vector(nt, 511)
    x_kt = synth.random_vector(nt, 512)
    X = {"G": torch.tensor(x_g, device=dev), "GT": torch.tensor(x_gt, device=dev),
         "K": torch.tensor(x_k, device=dev), "KT": torch.tensor(x_kt, device=dev)}
    Y = {"G": torch.zeros(nt, dtype=torch.float64, device=dev),
         "GT": torch.zeros(nt, dtype=torch.float64, device=dev),
         "K": torch.zeros(nt, dtype=torch.float64, device=dev),
         "KT": torch.zeros(nv, dtype=torch.float64, device=dev)}
    PRODUCTS = (("G", "G", False), ("GT", "G", True), ("K", "K", False), ("KT", "K", True))

    def step_items(suffix):
        return [(ops[o + suffix], X[p], Y[p], tr) for p, o, tr in PRODUCTS]

    # one clean product of each for accuracy
    def single(op, p, tr):
        out = torch.zeros_like(Y[p])
        op.matvec(X[p], out, trans=tr)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    y = {}
    for suffix in ("", "32") if not args.no_mixed else ("",):
        for p, o, tr in PRODUCTS:
            y[p + suffix] = single(ops[o + suffix], p, tr)

    ms64, ph64 = time_steps(torch, step_items(""), args.steps, args.warmup)
    log("FP64 step (G x, G^T x, K x, K^T x): %.3f ms" % ms64)
    if not args.no_mixed:
        ms32, ph32 = time_steps(torch, step_items("32"), args.steps, args.warmup)
        log("mixed step: %.3f ms" % ms32)

    # per-operator detail: phases (mean over the operator's A x and A^T x in
    # the timed steps) and each product timed alone
    detail = {}
    dominant = None
    step_bytes = {"": 0, "32": 0}
    for name, ph in (("G", ph64[0]), ("K", ph64[1])) + ((("G32", ph32[0]), ("K32", ph32[1]))
                                                         if not args.no_mixed else ()):
        inf = ops[name].info()
        fsz = 4 if name.endswith("32") else 8
        b, bt = alg_bytes(inf, fsz), alg_bytes(inf, fsz, trans=True)
        suffix = "32" if name.endswith("32") else ""
        base = name[0]
        t_a = time_product(torch, ops[name], X[base], Y[base], False)
        t_t = time_product(torch, ops[name], X[base + "T"], Y[base + "T"], True)
        step_bytes[suffix] += b["total"] + bt["total"]
        d = dict(ms_Ax=t_a, ms_ATx=t_t, gbps_Ax=b["total"] / t_a / 1e6, gbps_ATx=bt["total"] / t_t / 1e6,
                 phases_ms=ph, alg_bytes_Ax=b["total"], alg_bytes_ATx=bt["total"],
                 coupling_gbps=b["coupling"] / ph["coupling"] / 1e6,
                 near_gbps=b["near"] / ph["nearfield"] / 1e6,
                 bytes_near=inf["bytes_near"], bytes_far=inf["bytes_far"],
                 bytes_transposed=inf["bytes_transposed"],
                 nfar=inf["nfar"], nnear=inf["nnear"], assembly_s=assembly_s[name],
                 mean_rank=(inf["mean_rank_row"], inf["mean_rank_col"]),
                 max_rank=(inf["max_rank_row"], inf["max_rank_col"]))
        detail[name] = d
        log("%s: A x %.3f ms (%.0f GB/s), A^T x %.3f ms (%.0f GB/s)" % (name, t_a, d["gbps_Ax"], t_t,
                                                                        d["gbps_ATx"]))
        if not suffix:
            for kname, ms_k, by in (("coupling", ph["coupling"], b["coupling"]),
                                    ("nearfield", ph["nearfield"], b["near"])):
                if dominant is None or ms_k > dominant[2]:
                    dominant = (name, kname, ms_k, by)
    if not args.no_mixed:
        for p, o, tr in PRODUCTS:
            a, r = y[p + "32"], y[p]
            detail[o + "32"]["rel_diff_vs_fp64" + ("_T" if tr else "")] = float(
                np.linalg.norm(a - r) / np.linalg.norm(r))
    traffic_config = {"s": args.s, "leaf": args.leaf, "order": args.order, "q_near": args.q_near,
                      "tol": args.tol}
    # measured read ceiling of this GPU: torch's sum over 8 GiB of doubles
    buf = torch.ones(1 << 30, dtype=torch.float64, device=dev)
    for _ in range(2):
        buf.sum()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        buf.sum()
    torch.cuda.synchronize()
    read_gbps = 8 * (1 << 30) * 5 / (time.perf_counter() - t0) / 1e9
    del buf
    torch.cuda.empty_cache()
    log("read ceiling (torch sum over 8 GiB): %.0f GB/s" % read_gbps)
    # the same kernel with every phase on one stream (no overlap with the far field)
    dop = ops[dominant[0]]
    dop.set_overlap(False)
    solo_ms, solo_ph = time_steps(torch, [(dop, X[dominant[0]], Y[dominant[0]], False),
                                          (dop, X[dominant[0] + "T"], Y[dominant[0] + "T"], True)],
                                  max(3, args.steps // 4), 1)
    dop.set_overlap(True)
    solo_k = solo_ph[0][dominant[1]]
    log("%s %s alone: %.3f ms per launch (%.0f GB/s)" % (dominant[0], dominant[1], solo_k,
                                                         dominant[3] / solo_k / 1e6))

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
            "workload": "unit sphere (octahedron split s=%d, %d triangles, %d vertices): G x, G^T x, "
                        "K x and K^T x per step, H^2 Chebyshev order %d recompressed to %g, leaf %d, "
                        "eta 1, q_near %d" % (args.s, nt, nv, args.order, args.tol, args.leaf, args.q_near),
            "triangles": nt, "vertices": nv, "order_m": args.order, "leaf": args.leaf,
            "q_near": args.q_near, "recompress_tol": args.tol, "x_seeds": [501, 511, 502, 512],
        },
        "step_gbps": round(step_bytes[""] / ms64 / 1e6, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": kernel_name(dominant[0], dominant[1], ops[dominant[0]].info()),
            "achieved": round(dominant[3] / dominant[2] / 1e6, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(dominant[3] / dominant[2] / 1e6 / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic("%s %s" % dominant[:2], traffic_config),
            "alg_bytes": dominant[3],
            "avg_launch_ms": round(dominant[2], 4),
            "concurrent": "the nearfield runs on its own stream beside the far-field kernels, so its "
                          "launches share HBM with them; step_gbps is the whole step's rate",
            "solo": {"avg_launch_ms": round(solo_k, 4),
                     "achieved": round(dominant[3] / solo_k / 1e6, 1),
                     "frac": round(dominant[3] / solo_k / 1e6 / HBM_PEAK_GBS, 4),
                     "note": "same launches with every phase on one stream (h2b_op_set_overlap 0), "
                             "timed after the step"},
            "measured_read_gbps": round(read_gbps, 1),
            "solo_frac_of_measured_read": round(dominant[3] / solo_k / 1e6 / read_gbps, 4),
        },
        "detail": detail,
    }
    if not args.no_mixed:
        out["mixed"] = {"ms_per_step": round(ms32, 4), "speedup_vs_fp64": round(ms64 / ms32, 3),
                        "rel_diff": {p: detail[o + "32"]["rel_diff_vs_fp64" + ("_T" if tr else "")]
                                     for p, o, tr in PRODUCTS},
                        "step_gbps": round(step_bytes["32"] / ms32 / 1e6, 1)}

    # accuracy on the 1,000 oracle rows stored for this workload, if present
    gold_path = os.path.join(ROOT, "tests", "golden", "sphere2M_oracle_rows.json")
    if (os.path.exists(gold_path) and args.s == 512 and args.q_near == 6 and args.order == 4
            and args.leaf == 64 and args.tol == 1e-6):
        with open(gold_path) as fh:
            gold = json.load(fh)
        rows = np.asarray(gold["rows"])
        acc1000 = {}
        for name in ops:
            ref = np.asarray(gold[name[0]]["y"])
            got = y[name][rows]
            acc1000[name] = {"rel_2norm": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                             "max_row_over_max": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))}
        out["oracle_rows_1000"] = acc1000
        log("1,000 stored oracle rows: " + ", ".join("%s %.3e" % (k, v["rel_2norm"]) for k, v in acc1000.items()))

    if not args.no_solve:
        out["dtn_solve"] = dtn_solve(torch, h2b, ops, verts, tris, ("", "32") if not args.no_mixed else ("",),
                                     {"": detail["G"]["ms_Ax"],
                                      "32": detail["G32"]["ms_Ax"] if not args.no_mixed else None})
        out["ntd_solve"] = ntd_solve(torch, h2b, ops, verts, tris)

    if not args.no_batching:
        out["batching"] = batching(torch, h2b, synth, max(5, args.steps // 2))

    if not args.no_hchol:
        out["hchol_solve"] = hchol_solves(torch, h2b, [(64, 5e-3), (128, 2e-3)])

    if not args.no_gca_solve:
        # the benchmark operators make room for the GCA pair
        dop = None
        ops.clear()
        torch.cuda.empty_cache()
        try:
            out["gca_solve"] = gca_solve(torch, h2b, mesh, verts, tris, args)
        except (h2b.H2BError, RuntimeError, MemoryError) as e:
            out["gca_solve"] = {"error": str(e)}
            log("GCA solves failed: %s" % e)

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
        sample = {"G": np.sort(rng.choice(nt, nrows, replace=False)),
                  "K": np.sort(rng.choice(nt, nrows, replace=False))}
        xin = {"G": x_g, "K": x_k}
        log("oracle: %d rows of each of G and K on %d threads" % (nrows, nthreads))
        cb = cpu_baseline(verts, tris, args.q_near, sample, xin)
        # G^T x and K^T x evaluate the same pair integrals as G x and K x; they
        # are counted at the sampled cost of G x and K x (for K^T x a lower
        # bound: the oracle's vertex rows evaluate each pair once per vertex)
        est_ms = 2 * sum(cb["t"][p] / nrows * nt for p in sample) * 1e3
        log("oracle rows: " + ", ".join("%s %.1f s" % (p, cb["t"][p]) for p in sample))
        out["cpu_baseline"] = {
            "value": est_ms, "unit": "ms", "cores": cb["threads"], "kind": "oracle",
            "sample": "%d rows each of G and K (seed 503) of the same 2M-triangle operators, dense FP64 "
                      "quadrature, timed %.1f s + %.1f s and scaled by n/rows to one dense G x + K x; "
                      "G^T x and K^T x counted at the same cost (same pair integrals)"
                      % (nrows, cb["t"]["G"], cb["t"]["K"]),
        }
        acc = {}
        for suffix in ("", "32") if not args.no_mixed else ("",):
            for p in sample:
                got = y[p + suffix][sample[p]]
                acc[p + suffix] = float(np.linalg.norm(got - cb["y"][p]) / np.linalg.norm(cb["y"][p]))
        out["sampled_row_rel_err"] = acc
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
