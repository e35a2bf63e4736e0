"""GPU parity of batched products against the oracle.

Sixteen meshes of the many-meshes workload (spheres of random radius and
ellipsoids of random semi-axes, s ~ U{16..64}, i.e. 2,048 to 32,768
triangles), each with a block of 64 right-hand sides, run as one batch; the
rows sampled from every mesh equal the oracle's H^2 rows (same trees, same
interpolation; written out block by block without transfer matrices) to
rounding.
"""
import numpy as np
import pytest

import synth
from oracle import h2

pytestmark = pytest.mark.gpu


def _meshes(n=16, seed=302):
    """The many-meshes workload: even k a sphere of radius r ~ U[0.5, 2],
    odd k an ellipsoid with semi-axes ~ U[0.5, 2], s ~ U{16..64}."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        s = int(rng.integers(16, 65))
        if k % 2 == 0:
            r = rng.uniform(0.5, 2.0)
            out.append(synth.ellipsoid(s, r, r, r))
        else:
            a, b, c = rng.uniform(0.5, 2.0, size=3)
            out.append(synth.ellipsoid(s, a, b, c))
    return out


def test_batch_of_uneven_meshes_64_rhs_against_oracle_rows():
    import torch
    import paper_2001_05523_amd as h
    assert torch.cuda.is_available()
    leaf, m, q = 32, 4, 4
    meshes = _meshes()
    items, kernels = [], []
    for k, (v, t) in enumerate(meshes):
        kernel = "slp" if k % 3 else "dlp"
        op = h.Operator(v, t, kernel=kernel, leaf=leaf, order_m=m, q_near=q)
        X = torch.tensor(synth.random_vector(op.shape[1], 303 + k, cols=64), device="cuda").t().contiguous().t()
        Y = torch.zeros((64, op.shape[0]), dtype=torch.float64, device="cuda").t()
        items.append((op, X, Y))
        kernels.append(kernel)
    print("batch of %d meshes, %d triangles" % (len(items), sum(len(t) for _, t in meshes)), flush=True)
    batch = h.Batch(items, alpha=0.5)
    torch.cuda.synchronize()
    for rep in range(2):
        for _, _, Y in items:
            Y.zero_()
        torch.cuda.synchronize()
        batch.launch()
        torch.cuda.synchronize()
        if rep == 0:
            got = [Y.cpu().numpy().copy() for _, _, Y in items]
        else:
            for g, (_, _, Y) in zip(got, items):
                assert np.array_equal(g, Y.cpu().numpy())
    rng = np.random.default_rng(304)
    for k, ((v, t), kernel, (op, X, _)) in enumerate(zip(meshes, kernels, items)):
        rows = np.sort(rng.choice(len(t), 2, replace=False))
        ref = 0.5 * h2.h2_rows(v, t, kernel, leaf, m, rows, X.cpu().numpy(), q_near=q)
        d = np.max(np.abs(got[k][rows] - ref)) / np.max(np.abs(ref))
        print("mesh %d (%s, %d triangles): max rel diff to oracle rows %.2e" % (k, kernel, len(t), d), flush=True)
        assert d <= 1e-11, (k, d)


def _eager_vs_batch(h, torch, items, alpha, trans):
    refs = []
    for op, X, Y in items:
        R = torch.zeros_like(Y)
        op.matvec(X, R, alpha=alpha, trans=trans)
        refs.append(R)
    batch = h.Batch(items, alpha=alpha, trans=trans)
    for rep in range(3):
        for _, _, Y in items:
            Y.zero_()
        torch.cuda.synchronize()
        batch.launch()
        torch.cuda.synchronize()
        for (_, _, Y), R in zip(items, refs):
            scale = float(R.abs().max())
            assert float((Y - R).abs().max()) <= 1e-12 * scale
        # eager work between replays
        items[0][0].matvec(items[0][1], refs[0], alpha=0.0, trans=trans)
        torch.cuda.synchronize()
    return batch


@pytest.mark.parametrize("trans", [False, True])
def test_merged_batch_single_vectors_match_eager(trans):
    """One vector per mesh, FP64, A x and A^T x (the transposed copies): the
    merged batch (one launch per step for all meshes) equals the eager
    products on every replay."""
    import torch
    import paper_2001_05523_amd as h
    items = []
    for k, (v, t) in enumerate(_meshes(8, seed=305)):
        op = h.Operator(v, t, kernel="slp" if k % 2 else "dlp", leaf=32, order_m=3, q_near=4)
        nin = op.shape[0] if trans else op.shape[1]
        nout = op.shape[1] if trans else op.shape[0]
        X = torch.tensor(synth.random_vector(nin, 306 + k), device="cuda")
        items.append((op, X, torch.zeros(nout, dtype=torch.float64, device="cuda")))
    _eager_vs_batch(h, torch, items, -0.5, trans)


def test_mixed_batch_falls_back_to_per_operator_graph():
    """Operators whose products differ (here the number of right-hand sides)
    cannot share one merged program; the batch then captures each operator's
    product as its own branch and still equals the eager products."""
    import torch
    import paper_2001_05523_amd as h
    items = []
    for k, (v, t) in enumerate(_meshes(4, seed=307)):
        op = h.Operator(v, t, kernel="slp", leaf=32, order_m=3, q_near=4)
        nr = 1 if k % 2 else 8
        if nr == 1:
            X = torch.tensor(synth.random_vector(op.shape[1], 308 + k), device="cuda")
            Y = torch.zeros(op.shape[0], dtype=torch.float64, device="cuda")
        else:
            X = torch.tensor(synth.random_vector(op.shape[1], 308 + k, cols=nr), device="cuda").t().contiguous().t()
            Y = torch.zeros((nr, op.shape[0]), dtype=torch.float64, device="cuda").t()
        items.append((op, X, Y))
    _eager_vs_batch(h, torch, items, 1.0, False)
