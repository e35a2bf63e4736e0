"""Shape gradient of b = x^T G y with respect to the vertex coordinates (the
differentiation form): the library's adjoint kernels against central finite
differences of the same frozen-structure H^2 form, against finite
differences of the dense oracle, and through torch.autograd."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _lib():
    import paper_2001_05523_amd as h
    return h


def _form(op, x, y):
    torch = _torch()
    gy = torch.zeros_like(x)
    op.matvec(y, gy)
    torch.cuda.synchronize()
    return float(torch.dot(x, gy))


def _fd(op, verts, x, y, v, d, h):
    vp = verts.copy()
    vp[v, d] += h
    op.set_geometry(vp)
    fp = _form(op, x, y)
    vp[v, d] -= 2 * h
    op.set_geometry(vp)
    fm = _form(op, x, y)
    op.set_geometry(verts)
    return (fp - fm) / (2 * h)


def test_adjoint_matches_finite_differences_small():
    torch = _torch()
    h2b = _lib()
    verts, tris = synth.perturbed_sphere(8, 401)
    op = h2b.Operator(verts, tris, kernel="slp", leaf=16, order_m=3, q_near=4)
    x = torch.tensor(synth.random_vector(len(tris), 402), device="cuda")
    y = torch.tensor(synth.random_vector(len(tris), 403), device="cuda")
    g = op.shape_grad(x, y).cpu().numpy()
    rng = np.random.default_rng(404)
    scale = np.abs(g).max()
    for v in rng.choice(len(verts), 12, replace=False):
        for d in range(3):
            fd = _fd(op, verts, x, y, v, d, 1e-6)
            assert abs(fd - g[v, d]) <= 1e-6 * scale, (v, d, fd, g[v, d])


def test_adjoint_close_to_dense_oracle_gradient():
    """The oracle's gradient (central differences of the dense Galerkin form,
    h = 1e-6) agrees with the H^2 adjoint to within the interpolation error."""
    torch = _torch()
    h2b = _lib()
    verts, tris = synth.perturbed_sphere(8, 401)
    q = 4
    op = h2b.Operator(verts, tris, kernel="slp", leaf=16, order_m=4, q_near=q)
    xn = synth.random_vector(len(tris), 402)
    yn = synth.random_vector(len(tris), 403)
    x = torch.tensor(xn, device="cuda")
    y = torch.tensor(yn, device="cuda")
    g = op.shape_grad(x, y).cpu().numpy()
    rng = np.random.default_rng(405)
    scale = np.abs(g).max()
    errs = []
    for v in rng.choice(len(verts), 12, replace=False):
        for d in range(3):
            vp = verts.copy()
            vp[v, d] += 1e-6
            fp = xn @ oracle.slp_dense(vp, tris, q) @ yn
            vp[v, d] -= 2e-6
            fm = xn @ oracle.slp_dense(vp, tris, q) @ yn
            errs.append(abs((fp - fm) / 2e-6 - g[v, d]) / scale)
    print("max |adjoint - oracle FD| / max|grad| = %.3e" % max(errs))
    # the H^2 form differs from the dense one by the order-4 interpolation
    # error of the far field (about 1e-4 of the gradient on this mesh)
    assert max(errs) <= 5e-4


@pytest.mark.parametrize("s,nvert", [(4, None), (8, 16)])
def test_adjoint_equals_dense_oracle_gradient_without_far_field(s, nvert):
    """Far field disabled, so x^T G y is the dense Galerkin form of the
    oracle: the adjoint gradient must equal central differences of the
    oracle's dense matrix (same quadrature, h = 1e-6) up to the difference
    error, at every vertex of the 128-triangle sphere and at 16 vertices of
    the 512-triangle one.  A central difference of a form of size |b| in
    FP64 carries about eps |b| / h ~ 1e-10 |b| of rounding, plus h^2 terms."""
    torch = _torch()
    h2b = _lib()
    verts, tris = synth.perturbed_sphere(s, 401 + s)
    q = 4
    op = h2b.Operator(verts, tris, kernel="slp", leaf=16, q_near=q, far_disabled=True)
    xn = synth.random_vector(len(tris), 412)
    yn = synth.random_vector(len(tris), 413)
    g = op.shape_grad(torch.tensor(xn, device="cuda"), torch.tensor(yn, device="cuda")).cpu().numpy()
    scale = np.abs(g).max()
    rng = np.random.default_rng(414)
    vs = range(len(verts)) if nvert is None else rng.choice(len(verts), nvert, replace=False)
    err = 0.0
    for v in vs:
        for d in range(3):
            vp = verts.copy()
            vp[v, d] += 1e-6
            fp = xn @ oracle.slp_dense(vp, tris, q) @ yn
            vp[v, d] -= 2e-6
            fm = xn @ oracle.slp_dense(vp, tris, q) @ yn
            err = max(err, abs((fp - fm) / 2e-6 - g[v, d]) / scale)
    print("s=%d: max |adjoint - oracle FD| / max|grad| = %.3e" % (s, err))
    assert err <= 1e-7


def test_autograd_function():
    torch = _torch()
    h2b = _lib()
    verts, tris = synth.perturbed_sphere(8, 401)
    op = h2b.Operator(verts, tris, kernel="slp", leaf=16, order_m=3, q_near=4)
    V = torch.tensor(verts, requires_grad=True)
    x = torch.tensor(synth.random_vector(len(tris), 402), device="cuda", requires_grad=True)
    y = torch.tensor(synth.random_vector(len(tris), 403), device="cuda", requires_grad=True)
    b = h2b.SlpBilinear.apply(V, x, y, op)
    b.backward()
    torch.cuda.synchronize()
    g = op.shape_grad(x.detach(), y.detach()).cpu()
    assert torch.allclose(V.grad.cpu(), g, rtol=0, atol=1e-12 * float(g.abs().max()))
    gy = torch.zeros_like(x)
    op.matvec(y.detach(), gy)
    gtx = torch.zeros_like(y)
    op.matvec(x.detach(), gtx, trans=True)
    assert torch.allclose(x.grad, gy) and torch.allclose(y.grad, gtx)


def test_perturbed_sphere_131k_adjoint_vs_finite_differences():
    """Perturbed sphere of 131,072 triangles (r = 1 + 0.1 sum_{l<=8} c_lm Y_lm),
    order 4, leaf 64, q_near 5: adjoint against central differences (h = 1e-6,
    FP64, frozen structure) on 100 random vertices x 3 coordinates."""
    torch = _torch()
    h2b = _lib()
    verts, tris = synth.perturbed_sphere(128, 401)
    op = h2b.Operator(verts, tris, kernel="slp", leaf=64, order_m=4, q_near=5)
    x = torch.tensor(synth.random_vector(len(tris), 402), device="cuda")
    y = torch.tensor(synth.random_vector(len(tris), 403), device="cuda")
    g = op.shape_grad(x, y).cpu().numpy()
    scale = np.abs(g).max()
    rng = np.random.default_rng(404)
    worst = 0.0
    for v in rng.choice(len(verts), 100, replace=False):
        for d in range(3):
            fd = _fd(op, verts, x, y, v, d, 1e-6)
            worst = max(worst, abs(fd - g[v, d]) / scale)
    print("max |adjoint - FD| / max|grad| = %.3e" % worst)
    assert worst <= 1e-5
