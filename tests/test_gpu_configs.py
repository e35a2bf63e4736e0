"""Parity at the benchmark configurations, on outputs the oracle can compute
row by row (sampled rows of the dense Galerkin products).

* 32,768-triangle sphere, G and K, order 4 recompressed to 1e-6, leaf 32,
  q_near 4: FP64 and FP32 far field.
* 2,097,152-triangle sphere, order 4 recompressed to 1e-6, leaf 64, q_near 6,
  in the launch configuration bench.py times; and the Green cross
  approximation of the same operators against the stored oracle rows.

The H^2 error against the dense matrix is the interpolation error of order 4.
For K it grows like 1/h at fixed order: on a smooth surface <x - y, n_y> is
O(r^2), so the kernel's cancellation amplifies the error of the
differentiated interpolant.  The bounds below are those errors with margin;
exact parity is pinned at small sizes against the oracle's H^2 matrix."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _product(op, x, trans=False):
    torch = _torch()
    X = torch.tensor(x, device="cuda")
    Y = torch.zeros(op.shape[1] if trans else op.shape[0], dtype=torch.float64, device="cuda")
    op.matvec(X, Y, trans=trans)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_sphere_32k_sampled_rows(dtype):
    import paper_2001_05523_amd as h2b
    v, t = synth.octa_sphere(64)
    rng = np.random.default_rng(203)
    out = {}
    for kernel, seed, bound in (("slp", 201, 1e-3), ("dlp", 202, 2e-2)):
        op = h2b.Operator(v, t, kernel=kernel, leaf=32, order_m=4, q_near=4, recompress_tol=1e-6,
                          farfield_dtype=dtype)
        x = synth.random_vector(op.shape[1], seed)
        y = _product(op, x)
        rows = np.sort(rng.choice(len(t), 24, replace=False))
        ref = (oracle.slp_rows if kernel == "slp" else oracle.dlp_rows)(v, t, 4, rows, x)
        out[kernel] = _rel(y[rows], ref)
        # transposed product on sampled columns
        xt = synth.random_vector(op.shape[0], seed + 10)
        yt = _product(op, xt, trans=True)
        cols = np.sort(rng.choice(op.shape[1], 8, replace=False))
        reft = (oracle.slp_rows if kernel == "slp" else oracle.dlp_rows)(v, t, 4, cols, xt, trans=True)
        out[kernel + "T"] = _rel(yt[cols], reft)
        print(kernel, dtype, "sampled-row error %.3e, transposed %.3e, mean rank %.1f"
              % (out[kernel], out[kernel + "T"], op.info()["mean_rank_row"]))
        assert out[kernel] <= bound and out[kernel + "T"] <= bound


def test_sphere_2M_sampled_rows():
    import paper_2001_05523_amd as h2b
    v, t = synth.octa_sphere(512)
    rng = np.random.default_rng(503)
    mesh = h2b.Mesh(v, t)
    for kernel, seed, bound in (("slp", 501, 1e-3), ("dlp", 502, 5e-2)):
        op = h2b.Operator(mesh=mesh, kernel=kernel, leaf=64, order_m=4, q_near=6, recompress_tol=1e-6)
        x = synth.random_vector(op.shape[1], seed)
        y = _product(op, x)
        del op
        rows = np.sort(rng.choice(len(t), 16, replace=False))
        ref = (oracle.slp_rows if kernel == "slp" else oracle.dlp_rows)(v, t, 6, rows, x)
        err = _rel(y[rows], ref)
        print(kernel, "2M sampled-row error %.3e" % err)
        assert err <= bound


GOLDEN_2M = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sphere2M_oracle_rows.json")


@pytest.mark.skipif(not os.path.exists(GOLDEN_2M), reason="oracle rows not generated (tests/golden/sphere2M_oracle_rows.py)")
def test_sphere_2M_1000_oracle_rows():
    """1,000 rows of G x and K x on the 2,097,152-triangle sphere (order 4
    recompressed to 1e-6, leaf 64, q_near 6), FP64 and FP32 far field, against
    the oracle's dense rows stored by tests/golden/sphere2M_oracle_rows.py.
    The error is the order-4 interpolation error; the FP32 far field adds at
    most 1e-5 to it."""
    import json
    import paper_2001_05523_amd as h2b
    with open(GOLDEN_2M) as fh:
        gold = json.load(fh)
    v, t = synth.octa_sphere(512)
    rows = np.asarray(gold["rows"])
    mesh = h2b.Mesh(v, t)
    for name, kernel, bound in (("G", "slp", 1e-3), ("K", "dlp", 5e-2)):
        ref = np.asarray(gold[name]["y"])
        x = synth.random_vector(len(t) if kernel == "slp" else len(v), gold[name]["x_seed"])
        errs = {}
        for dtype in ("f64", "f32"):
            op = h2b.Operator(mesh=mesh, kernel=kernel, leaf=64, order_m=4, q_near=gold["q_near"],
                              recompress_tol=1e-6, farfield_dtype=dtype)
            y = _product(op, x)
            del op
            errs[dtype] = _rel(y[rows], ref)
            print(name, dtype, "1000-row error %.3e, max row error / max|y| %.3e"
                  % (errs[dtype], np.max(np.abs(y[rows] - ref)) / np.max(np.abs(ref))))
            assert errs[dtype] <= bound
        assert abs(errs["f32"] - errs["f64"]) <= 1e-5


@pytest.mark.skipif(not os.path.exists(GOLDEN_2M), reason="stored oracle rows not generated")
def test_sphere_2M_gca_1000_oracle_rows():
    """The same 1,000 stored oracle rows against the Green cross
    approximation of G and K (order 4 per face direction, tolerance 1e-6), as
    built and with its bases recompressed to 1e-6: GCA reaches the accuracy
    that order-4 interpolation cannot (all within 1e-5; measured 1.4e-6 as
    built and 3-4e-6 recompressed, against 2.5e-4 and 2.0e-2), and the
    recompression shrinks its far field at least threefold."""
    import json
    import paper_2001_05523_amd as h2b
    with open(GOLDEN_2M) as fh:
        gold = json.load(fh)
    v, t = synth.octa_sphere(512)
    rows = np.asarray(gold["rows"])
    mesh = h2b.Mesh(v, t)
    for name, kernel, bound in (("G", "slp", 1e-5), ("K", "dlp", 1e-5)):
        ref = np.asarray(gold[name]["y"])
        x = synth.random_vector(len(t) if kernel == "slp" else len(v), gold[name]["x_seed"])
        far = {}
        for rc in (0.0, 1e-6):
            op = h2b.Operator(mesh=mesh, kernel=kernel, leaf=64, order_m=4, q_near=gold["q_near"], gca_tol=1e-6,
                              recompress_tol=rc, transposed_copy=False)
            y = _product(op, x)
            far[rc] = op.info()["bytes_far"]
            del op
            err = _rel(y[rows], ref)
            print(name, "GCA (recompressed to %g) 1000-row error %.3e, far field %.2f GB" % (rc, err, far[rc] / 1e9))
            assert err <= bound
        assert far[1e-6] * 3 <= far[0.0]
