"""Host-side checks of the C-ABI library (no GPU needed): every declared
symbol is exported, the trees and block lists equal the oracle's (integer and
index work, bit-exact), and invalid input is rejected before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import h2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2001_05523_amd as h
    return h


def test_header_symbols_exported():
    h = _lib()
    text = open(os.path.join(ROOT, "include", "h2bem.h")).read()
    decl = set(re.findall(r"\b(h2b_[a-z_0-9]+)\s*\(", text))
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(h._lib, name), name
    assert decl == set(h.EXPORTED)


@pytest.mark.parametrize("space,leaf,s", [(0, 32, 8), (1, 16, 8), (0, 8, 4), (1, 5, 4), (0, 64, 16)])
def test_cluster_tree_equals_oracle(space, leaf, s):
    h = _lib()
    v, t = synth.octa_sphere(s)
    T = h.Tree(h.Mesh(v, t), space, leaf)
    a = T.arrays()
    pts = v[t].mean(axis=1) if space == 0 else v
    _, perm, cl = h2.cluster_tree(pts, leaf)
    h2.support_boxes(cl, v, t, "P0" if space == 0 else "P1")
    assert T.nclusters == len(cl)
    np.testing.assert_array_equal(a["perm"], perm)
    np.testing.assert_array_equal(a["begin"], [c.begin for c in cl])
    np.testing.assert_array_equal(a["end"], [c.end for c in cl])
    np.testing.assert_array_equal(a["box"], np.array([np.r_[c.lo, c.hi] for c in cl]))


@pytest.mark.parametrize("kernel,leaf,s", [("slp", 32, 8), ("slp", 16, 16), ("dlp", 16, 16),
                                           ("dlp", 8, 8)])
def test_block_lists_equal_oracle(kernel, leaf, s):
    h = _lib()
    v, t = synth.octa_sphere(s)
    m = h.Mesh(v, t)
    R = h.Tree(m, 0, leaf)
    C = R if kernel == "slp" else h.Tree(m, 1, leaf)
    B = h.Blocks(R, C, 1.0)
    far, near = B.lists()
    _, _, rcl = h2.cluster_tree(v[t].mean(axis=1), leaf)
    h2.support_boxes(rcl, v, t, "P0")
    if kernel == "slp":
        ccl = rcl
    else:
        _, _, ccl = h2.cluster_tree(v, leaf)
        h2.support_boxes(ccl, v, t, "P1")
    f, n = h2.block_tree(rcl[0], ccl[0], 1.0)
    np.testing.assert_array_equal(far.reshape(-1, 2), np.array([(a.id, b.id) for a, b in f]).reshape(-1, 2))
    np.testing.assert_array_equal(near, np.array([(a.id, b.id) for a, b in n]))
    ne = sum((a.end - a.begin) * (b.end - b.begin) for a, b in n)
    assert B.near_entries == ne


def test_far_disabled_gives_only_near_blocks():
    h = _lib()
    v, t = synth.octa_sphere(8)
    m = h.Mesh(v, t)
    R = h.Tree(m, 0, 32)
    B = h.Blocks(R, R, 1.0, far_disabled=True)
    assert B.nfar == 0
    assert B.near_entries == len(t) ** 2


def test_invalid_meshes_rejected():
    h = _lib()
    v, t = synth.octa_sphere(2)
    bad = t.copy()
    bad[3, 1] = len(v)
    with pytest.raises(h.H2BError) as e:
        h.Mesh(v, bad)
    assert e.value.code == h.H2B_EINVAL and "out of range" in str(e.value)
    bad = t.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(h.H2BError):
        h.Mesh(v, bad)
    vv = v.copy()
    vv[t[2, 2]] = vv[t[2, 0]]
    with pytest.raises(h.H2BError) as e:
        h.Mesh(vv, t)
    assert "zero area" in str(e.value)
    vv = v.copy()
    vv[0, 0] = np.nan
    with pytest.raises(h.H2BError):
        h.Mesh(vv, t)


def test_invalid_tree_and_block_arguments():
    h = _lib()
    v, t = synth.octa_sphere(2)
    m = h.Mesh(v, t)
    with pytest.raises(h.H2BError):
        h.Tree(m, 0, 0)
    with pytest.raises(h.H2BError):
        h.Tree(m, 7, 4)
    R = h.Tree(m, 0, 4)
    C = h.Tree(m, 1, 4)
    with pytest.raises(h.H2BError):
        h.Blocks(R, C, 0.0)
    with pytest.raises(h.H2BError):
        h.Blocks(C, R, 1.0)  # rows must be the triangle tree
    other = h.Tree(h.Mesh(v, t), 0, 4)
    with pytest.raises(h.H2BError):
        h.Blocks(R, other, 1.0)


def _assemble_status(h, blocks, kernel, **kw):
    p = h.default_params(**kw)
    out = ctypes.c_void_p()
    return h.h2b_assemble(blocks.handle, kernel, ctypes.byref(p), None, ctypes.byref(out))


def test_assembly_arguments_rejected_on_the_host():
    """Requests that assembly refuses before any device call: the
    single-layer matrix on two different triangle trees (its column basis is
    the row basis), an FP32 or BF16 far field on non-orthonormal bases
    (interpolation without recompression, cross approximation) or with
    ranks above 64 recompressed into it, parameters out of range."""
    h = _lib()
    v, t = synth.octa_sphere(4)
    m = h.Mesh(v, t)
    R = h.Tree(m, 0, 8)
    R2 = h.Tree(m, 0, 16)
    C = h.Tree(m, 1, 8)
    assert _assemble_status(h, h.Blocks(R, R2, 1.0), h.H2B_SLP) == h.H2B_EINVAL
    assert b"one cluster tree" in h.h2b_last_error()
    assert _assemble_status(h, h.Blocks(R2, R, 1.0), h.H2B_SLP) == h.H2B_EINVAL
    B = h.Blocks(R, R, 1.0)
    BK = h.Blocks(R, C, 1.0)
    for dt in (h.H2B_F32, h.H2B_BF16):
        for blk, ker in ((B, h.H2B_SLP), (BK, h.H2B_DLP)):
            assert _assemble_status(h, blk, ker, farfield_dtype=dt) == h.H2B_ENOTSUP
            assert _assemble_status(h, blk, ker, farfield_dtype=dt, gca_tol=1e-4) == h.H2B_ENOTSUP
            assert b"orthonormal" in h.h2b_last_error()
    # ranks above 64 (cross approximation, orders 5-6) are recompressed in FP64 only
    assert _assemble_status(h, B, h.H2B_SLP, gca_tol=1e-4, recompress_tol=1e-6,
                            farfield_dtype=h.H2B_F32) == h.H2B_ENOTSUP
    assert _assemble_status(h, B, h.H2B_SLP, order_m=5, recompress_tol=1e-6,
                            farfield_dtype=h.H2B_F32) == h.H2B_ENOTSUP
    assert _assemble_status(h, B, h.H2B_SLP, order_m=7) == h.H2B_EINVAL
    assert _assemble_status(h, B, h.H2B_SLP, q_near=1) == h.H2B_EINVAL
    assert _assemble_status(h, B, h.H2B_DLP) == h.H2B_EINVAL  # K needs a P1 column tree
    assert _assemble_status(h, BK, h.H2B_SLP) == h.H2B_EINVAL


def test_allocator_failure_gives_enomem():
    """An installed allocator that returns NULL makes assembly fail with
    H2B_ENOMEM before any device work, with no handle written; exactly one
    NULL callback is rejected.  The allocator is restored afterwards."""
    h = _lib()
    calls = []

    def alloc(nbytes, stream, ctx):
        calls.append(nbytes)
        return None

    def free(ptr, stream, ctx):
        raise AssertionError("nothing was allocated")

    a, f = h._ALLOC_FN(alloc), h._FREE_FN(free)
    v, t = synth.octa_sphere(4)
    m = h.Mesh(v, t)
    R = h.Tree(m, 0, 8)
    B = h.Blocks(R, R, 1.0)
    try:
        assert h.h2b_set_allocator(a, h._FREE_FN(), None) == h.H2B_EINVAL
        assert h.h2b_set_allocator(h._ALLOC_FN(), f, None) == h.H2B_EINVAL
        assert h.h2b_set_allocator(a, f, None) == h.H2B_OK
        p = h.default_params()
        out = ctypes.c_void_p()
        assert h.h2b_assemble(B.handle, h.H2B_SLP, ctypes.byref(p), None, ctypes.byref(out)) == h.H2B_ENOMEM
        assert out.value is None
        assert b"returned NULL" in h.h2b_last_error()
        assert len(calls) == 1 and calls[0] > 0
    finally:
        h.use_torch_allocator()


def test_null_arguments_rejected():
    h = _lib()
    out = ctypes.c_void_p()
    assert h.h2b_tree_build(None, 0, 4, ctypes.byref(out)) == h.H2B_EINVAL
    assert b"NULL" in h.h2b_last_error()
    assert h.h2b_matvec(None, 0, 1.0, None, 1, None, 1, 1, None) == h.H2B_EINVAL


@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("m,eps", [(2, 1e-2), (3, 1e-4)])
def test_gca_pivots_equal_oracle(space, m, eps):
    """The library's host construction of the Green cross approximation picks
    the oracle's ranks and pivots cluster by cluster (perturbed sphere: no
    mirror symmetries, so no ties), for triangle clusters and for the vertex
    clusters of K's columns."""
    from oracle import gca, h2
    h = _lib()
    v, t = synth.perturbed_sphere(4, seed=3)
    mesh = h.Mesh(v, t)
    tree = h.Tree(mesh, space, 8)
    ranks, piv = tree.gca(m, eps)
    pts = v[t].mean(axis=1) if space == 0 else v
    root, perm, clusters = h2.cluster_tree(pts, 8)
    h2.support_boxes(clusters, v, t, "P0" if space == 0 else "P1")
    hat, _ = gca.gca_bases(v, t, clusters, perm, m, eps, space="P0" if space == 0 else "P1")
    assert len(clusters) == len(ranks)
    for c in clusters:
        assert ranks[c.id] == len(hat[c.id]), c.id
        assert np.array_equal(piv[c.id], hat[c.id]), c.id
    with pytest.raises(h.H2BError):
        tree.gca(0, eps)


def test_bench_runs_on_one_gpu_only():
    """bench.py measures one MI355X: a request for several GPUs exits with a
    message before touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_keyed_by_kernel_code():
    """The counter traffic in profiles/traffic.json is used only for the code
    it was measured on: the digest ignores comments and blank lines, changes
    with any code token, and matches the kernel sources in the tree."""
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src = b"int f(int a) { // add one\n  return a + 1; /* the\n  result */\n}\n\n"
    same = b"int f(int a) {\n\n  return a + 1;\n}\n"
    other = b"int f(int a) {\n  return a + 2;\n}\n"
    assert bench.code_text(src) == bench.code_text(same)
    assert bench.code_text(src) != bench.code_text(other)
    files = {"kernels.hip": src}
    read = lambda f: files.get(f, b"")
    d1 = bench.sources_digest(read)
    files["kernels.hip"] = same
    assert bench.sources_digest(read) == d1
    files["kernels.hip"] = other
    assert bench.sources_digest(read) != d1
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        assert json.load(fh)["sources_sha256"] == bench.sources_digest()
