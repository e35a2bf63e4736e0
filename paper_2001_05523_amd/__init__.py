"""Python binding of the gfx950 H^2 boundary element library (libh2bem.so).

Argument marshalling only: every step of the assembly and of the products runs
in the library's HIP kernels.  PyTorch supplies device memory (torch tensors
for x and y) and streams.  The functions keep the C names of include/h2bem.h;
``Mesh``, ``Tree``, ``Blocks`` and ``Operator`` are small owners of the handles.

Importing this package loads the library and fails loudly if it has not been
built (``python paper_2001_05523_amd/csrc/build_lib.py``).
"""
import ctypes
import os

import numpy as np

# torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch
# first makes the library bind to that same runtime, so device pointers and
# streams coming from torch are valid in the library: one process, one runtime.
import torch  # noqa: F401  (load order matters)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libh2bem.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libh2bem.so is not built: run `python paper_2001_05523_amd/csrc/build_lib.py` "
                      "(expected at %s)" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

H2B_OK, H2B_EINVAL, H2B_ENOMEM, H2B_EDEVICE, H2B_ESTATE, H2B_ENOTSUP = 0, -1, -2, -3, -4, -5
H2B_P0, H2B_P1 = 0, 1
H2B_SLP, H2B_DLP = 0, 1
H2B_F64, H2B_F32, H2B_BF16 = 0, 1, 2
_DTYPES = {"f64": H2B_F64, "f32": H2B_F32, "bf16": H2B_BF16}

_i64, _i32, _dbl, _vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
_P = ctypes.POINTER


class h2b_params(ctypes.Structure):
    _fields_ = [("order_m", ctypes.c_int), ("q_near", ctypes.c_int),
                ("recompress_tol", ctypes.c_double), ("farfield_dtype", ctypes.c_int),
                ("transposed_copy", ctypes.c_int), ("symmetric_near", ctypes.c_int), ("gca_tol", ctypes.c_double),
                ("recompute_coupling", ctypes.c_int)]


class h2b_op_stats(ctypes.Structure):
    _fields_ = [("rows", _i64), ("cols", _i64), ("nfar", _i64), ("nnear", _i64),
                ("near_entries", _i64), ("coupling_entries", _i64),
                ("row_basis_entries", _i64), ("col_basis_entries", _i64),
                ("bytes_near", _i64), ("bytes_far", _i64), ("bytes_vectors", _i64),
                ("row_coeffs", _i64), ("col_coeffs", _i64),
                ("max_rank_row", _i32), ("max_rank_col", _i32),
                ("mean_rank_row", _dbl), ("mean_rank_col", _dbl), ("bytes_transposed", _i64),
                ("near_sym_entries", _i64), ("near_sym_columns", _i64), ("near_sym_corrections", _i64),
                ("coupling_evals", _i64), ("cpl_sym_entries", _i64), ("cpl_sym_columns", _i64)]


class h2b_cg_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("check_every", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("zero_guess", ctypes.c_int), ("form", ctypes.c_int),
                ("precond", ctypes.c_int), ("hchol", _vp)]


class h2b_hchol_info(ctypes.Structure):
    _fields_ = [("n", _i64), ("eps", ctypes.c_double), ("coarse_entries", _i64), ("dense_entries", _i64),
                ("rk_entries", _i64), ("dense_blocks", _i64), ("rk_blocks", _i64), ("max_rank", ctypes.c_int),
                ("coarsened_blocks", _i64), ("converted_blocks", _i64), ("steps", _i64), ("tasks", _i64),
                ("convert_s", ctypes.c_double), ("coarsen_s", ctypes.c_double), ("factor_s", ctypes.c_double),
                ("upload_s", ctypes.c_double)]


class h2b_cg_result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("status", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]


H2B_CG_CONVERGED, H2B_CG_BREAKDOWN, H2B_CG_MAXITER = 1, 2, 3
H2B_FORM_PRODUCT, H2B_FORM_HYPERSINGULAR = 0, 1
_FORMS = {"product": H2B_FORM_PRODUCT, "hypersingular": H2B_FORM_HYPERSINGULAR}
H2B_PRECOND_NONE, H2B_PRECOND_BLOCK_JACOBI, H2B_PRECOND_HCHOL = 0, 1, 2
_PRECONDS = {None: H2B_PRECOND_NONE, "none": H2B_PRECOND_NONE, "block_jacobi": H2B_PRECOND_BLOCK_JACOBI,
             "hchol": H2B_PRECOND_HCHOL}
CG_STATUS = {H2B_CG_CONVERGED: "converged", H2B_CG_BREAKDOWN: "breakdown", H2B_CG_MAXITER: "max_iter"}


_SIGS = {
    "h2b_last_error": ([], ctypes.c_char_p),
    "h2b_version": ([], ctypes.c_char_p),
    "h2b_mesh_create": ([_i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _P(_vp)], ctypes.c_int),
    "h2b_mesh_destroy": ([_vp], ctypes.c_int),
    "h2b_tree_build": ([_vp, ctypes.c_int, ctypes.c_int, _P(_vp)], ctypes.c_int),
    "h2b_tree_destroy": ([_vp], ctypes.c_int),
    "h2b_tree_info": ([_vp, _P(_i64), _P(_i64), _P(_i64), _P(_i32)], ctypes.c_int),
    "h2b_tree_arrays": ([_vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "h2b_tree_gca": ([_vp, ctypes.c_int, _dbl, _vp, _vp, _P(_i64)], ctypes.c_int),
    "h2b_blocks_build": ([_vp, _vp, _dbl, ctypes.c_int, _P(_vp)], ctypes.c_int),
    "h2b_blocks_destroy": ([_vp], ctypes.c_int),
    "h2b_blocks_info": ([_vp, _P(_i64), _P(_i64), _P(_i64)], ctypes.c_int),
    "h2b_blocks_lists": ([_vp, _vp, _vp], ctypes.c_int),
    "h2b_params_default": ([_P(h2b_params)], None),
    "h2b_assemble": ([_vp, ctypes.c_int, _P(h2b_params), _vp, _P(_vp)], ctypes.c_int),
    "h2b_op_destroy": ([_vp], ctypes.c_int),
    "h2b_op_info": ([_vp, _P(h2b_op_stats)], ctypes.c_int),
    "h2b_matvec": ([_vp, ctypes.c_int, _dbl, _vp, _i64, _vp, _i64, ctypes.c_int, _vp], ctypes.c_int),
    "h2b_matvec_noalloc": ([_vp, ctypes.c_int, _dbl, _vp, _i64, _vp, _i64, ctypes.c_int, _vp], ctypes.c_int),
    "h2b_op_tune": ([_vp, ctypes.c_int, _vp, _P(_dbl)], ctypes.c_int),
    "h2b_batch_create": ([ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _P(_vp)], ctypes.c_int),
    "h2b_batch_launch": ([_vp, _vp], ctypes.c_int),
    "h2b_batch_destroy": ([_vp], ctypes.c_int),
    "h2b_op_set_geometry": ([_vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "h2b_slp_shape_grad": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "h2b_slp_bilinear": ([_vp, _vp, _vp, _vp, _vp, _vp], ctypes.c_int),
    "h2b_op_set_timing": ([_vp, ctypes.c_int], ctypes.c_int),
    "h2b_op_set_overlap": ([_vp, ctypes.c_int], ctypes.c_int),
    "h2b_op_phase_times": ([_vp, _vp], ctypes.c_int),
    "h2b_mass_matvec": ([_vp, ctypes.c_int, _dbl, _vp, _vp, _vp], ctypes.c_int),
    "h2b_cg_params_default": ([_P(h2b_cg_params)], None),
    "h2b_cg_solve": ([_vp, _vp, _vp, _P(h2b_cg_params), _P(h2b_cg_result), _vp, _vp], ctypes.c_int),
    "h2b_hypersingular_matvec": ([_vp, _dbl, _vp, _vp, _vp], ctypes.c_int),
    "h2b_hchol_build": ([_vp, _dbl, _P(_vp), _vp], ctypes.c_int),
    "h2b_hchol_from_dense": ([_vp, _vp, _dbl, _P(_vp)], ctypes.c_int),
    "h2b_hchol_solve_host": ([_vp, _vp, _vp], ctypes.c_int),
    "h2b_hchol_apply": ([_vp, _vp, _vp, _vp], ctypes.c_int),
    "h2b_hchol_get_info": ([_vp, _P(h2b_hchol_info)], ctypes.c_int),
    "h2b_hchol_destroy": ([_vp], ctypes.c_int),
}

_ALLOC_FN = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp, _vp)
_FREE_FN = ctypes.CFUNCTYPE(None, _vp, _vp, _vp)
_SIGS["h2b_set_allocator"] = ([_ALLOC_FN, _FREE_FN, _vp], ctypes.c_int)

EXPORTED = tuple(_SIGS)

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()[_name] = _f


# ------------------------------------------------------- device memory
#
# The library's device memory (operators, work vectors) comes from torch's
# caching allocator: it shows in torch.cuda.memory_allocated() and shares
# torch's pool.  The callbacks run with the GIL (ctypes takes it).

def _torch_alloc(nbytes, stream, ctx):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except RuntimeError:  # out of memory: the library reports H2B_ENOMEM
        return None


def _torch_free(ptr, stream, ctx):
    torch.cuda.caching_allocator_delete(int(ptr))


_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)


def use_torch_allocator():
    """Device memory of the library from torch's caching allocator (the
    default after import)."""
    _check(h2b_set_allocator(_TORCH_ALLOC, _TORCH_FREE, None))


def use_hip_allocator():
    """Device memory of the library from hipMalloc / hipFree."""
    _check(h2b_set_allocator(_ALLOC_FN(), _FREE_FN(), None))


# Handles still alive when the interpreter exits are not destroyed: their
# memory would go back to torch's allocator while torch itself is shutting
# down.  The process ends and the driver frees everything anyway.
_EXITING = [False]


def _at_exit():
    _EXITING[0] = True


import atexit  # noqa: E402
atexit.register(_at_exit)


class H2BError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("h2bem error %d: %s" % (code, msg))
        self.code = code


def _check(code):
    if code != H2B_OK:
        raise H2BError(code, _lib.h2b_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(_vp)


use_torch_allocator()


# --------------------------------------------------------------- handles

class Mesh:
    """Flat triangle mesh (host arrays copied into the library)."""

    def __init__(self, verts, tris):
        v = np.ascontiguousarray(np.asarray(verts, dtype=np.float64).reshape(-1, 3))
        t = np.ascontiguousarray(np.asarray(tris).reshape(-1, 3)).astype(np.int32)
        vx, vy, vz = (np.ascontiguousarray(v[:, d]) for d in range(3))
        t0, t1, t2 = (np.ascontiguousarray(t[:, d]) for d in range(3))
        h = _vp()
        _check(h2b_mesh_create(len(v), _ptr(vx), _ptr(vy), _ptr(vz), len(t),
                               _ptr(t0), _ptr(t1), _ptr(t2), ctypes.byref(h)))
        self.handle = h
        self.nv, self.nt = len(v), len(t)

    def __del__(self, _destroy=h2b_mesh_destroy, _exiting=_EXITING):
        if getattr(self, "handle", None) and not _exiting[0]:
            _destroy(self.handle)
            self.handle = None


class Tree:
    def __init__(self, mesh, space, leaf):
        h = _vp()
        _check(h2b_tree_build(mesh.handle, int(space), int(leaf), ctypes.byref(h)))
        self.handle = h
        n, nc, nl, lv = _i64(), _i64(), _i64(), _i32()
        _check(h2b_tree_info(h, ctypes.byref(n), ctypes.byref(nc), ctypes.byref(nl), ctypes.byref(lv)))
        self.n, self.nclusters, self.nleaves, self.nlevels = n.value, nc.value, nl.value, lv.value

    def arrays(self):
        perm = np.zeros(self.n, dtype=np.int32)
        b = np.zeros(self.nclusters, dtype=np.int32)
        e = np.zeros(self.nclusters, dtype=np.int32)
        par = np.zeros(self.nclusters, dtype=np.int32)
        box = np.zeros((self.nclusters, 6))
        _check(h2b_tree_arrays(self.handle, _ptr(perm), _ptr(b), _ptr(e), _ptr(par), _ptr(box)))
        return dict(perm=perm, begin=b, end=e, parent=par, box=box)

    def gca(self, order_m, eps):
        """Ranks (per cluster) and pivot lists of the Green cross
        approximation of this tree's bases, computed on the host."""
        ranks = np.zeros(self.nclusters, dtype=np.int32)
        piv = np.zeros(self.n * 2 + 12 * order_m * order_m * self.nclusters, dtype=np.int32)
        npiv = _i64()
        _check(h2b_tree_gca(self.handle, int(order_m), float(eps), _ptr(ranks), _ptr(piv), ctypes.byref(npiv)))
        piv = piv[:npiv.value]
        offs = np.concatenate([[0], np.cumsum(ranks)])
        return ranks, [piv[offs[c]:offs[c + 1]] for c in range(self.nclusters)]

    def __del__(self, _destroy=h2b_tree_destroy, _exiting=_EXITING):
        if getattr(self, "handle", None) and not _exiting[0]:
            _destroy(self.handle)
            self.handle = None


class Blocks:
    def __init__(self, rows, cols, eta=1.0, far_disabled=False):
        h = _vp()
        _check(h2b_blocks_build(rows.handle, cols.handle, float(eta), int(bool(far_disabled)),
                                ctypes.byref(h)))
        self.handle = h
        nf, nn, ne = _i64(), _i64(), _i64()
        _check(h2b_blocks_info(h, ctypes.byref(nf), ctypes.byref(nn), ctypes.byref(ne)))
        self.nfar, self.nnear, self.near_entries = nf.value, nn.value, ne.value

    def lists(self):
        far = np.zeros((self.nfar, 2), dtype=np.int32)
        near = np.zeros((self.nnear, 2), dtype=np.int32)
        _check(h2b_blocks_lists(self.handle, _ptr(far), _ptr(near)))
        return far, near

    def __del__(self, _destroy=h2b_blocks_destroy, _exiting=_EXITING):
        if getattr(self, "handle", None) and not _exiting[0]:
            _destroy(self.handle)
            self.handle = None


def default_params(**kw):
    p = h2b_params()
    h2b_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _vp(stream.cuda_stream)


class Operator:
    """Assembled H^2 approximation of G (kernel 'slp') or K ('dlp').

    ``op.matvec(x, y, alpha, trans)`` computes y += alpha op(A) x for torch
    float64 CUDA tensors x, y of shape (n,) or (n, nrhs) (column-major as
    produced by ``.t().contiguous().t()``, or nrhs = 1)."""

    def __init__(self, verts=None, tris=None, kernel="slp", leaf=32, order_m=4, q_near=4,
                 eta=1.0, far_disabled=False, recompress_tol=0.0, farfield_dtype="f64",
                 transposed_copy=True, symmetric_near=True, gca_tol=0.0, recompute_coupling=False, stream=None,
                 mesh=None):
        self.mesh = mesh if mesh is not None else Mesh(verts, tris)
        self.kernel = H2B_SLP if kernel == "slp" else H2B_DLP
        self.rows = Tree(self.mesh, H2B_P0, leaf)
        self.cols = self.rows if self.kernel == H2B_SLP else Tree(self.mesh, H2B_P1, leaf)
        self.blocks = Blocks(self.rows, self.cols, eta, far_disabled)
        p = default_params(order_m=order_m, q_near=q_near, recompress_tol=recompress_tol,
                           farfield_dtype=_DTYPES[farfield_dtype], transposed_copy=int(bool(transposed_copy)),
                           symmetric_near=int(bool(symmetric_near)), gca_tol=float(gca_tol),
                           recompute_coupling=int(bool(recompute_coupling)))
        h = _vp()
        _check(h2b_assemble(self.blocks.handle, self.kernel, ctypes.byref(p), _stream_ptr(stream),
                            ctypes.byref(h)))
        self.handle = h
        self.shape = (self.mesh.nt, self.mesh.nt if self.kernel == H2B_SLP else self.mesh.nv)

    def info(self):
        s = h2b_op_stats()
        _check(h2b_op_info(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def matvec(self, x, y, alpha=1.0, trans=False, stream=None):
        import torch
        nin = self.shape[0] if trans else self.shape[1]
        nout = self.shape[1] if trans else self.shape[0]
        for v, n, nm in ((x, nin, "x"), (y, nout, "y")):
            if not isinstance(v, torch.Tensor) or v.dtype != torch.float64 or not v.is_cuda:
                raise TypeError("%s must be a float64 CUDA tensor" % nm)
            if v.shape[0] != n:
                raise ValueError("%s has %d rows, expected %d" % (nm, v.shape[0], n))
        nrhs = 1 if x.dim() == 1 else x.shape[1]
        ldx = x.shape[0] if x.dim() == 1 else x.stride(1)
        ldy = y.shape[0] if y.dim() == 1 else y.stride(1)
        if x.dim() == 2 and x.stride(0) != 1 or y.dim() == 2 and y.stride(0) != 1:
            raise ValueError("x and y must be column-major")
        _check(h2b_matvec(self.handle, int(bool(trans)), float(alpha), _vp(x.data_ptr()), ldx,
                          _vp(y.data_ptr()), ldy, nrhs, _stream_ptr(stream)))
        return y

    def _product(self, x, trans):
        import torch
        if not isinstance(x, torch.Tensor) or x.dim() not in (1, 2):
            raise TypeError("x must be a 1-D or 2-D float64 CUDA tensor")
        nout = self.shape[1] if trans else self.shape[0]
        if x.dim() == 1:
            y = torch.zeros(nout, dtype=torch.float64, device=x.device)
        else:
            if x.stride(0) != 1:
                x = x.t().contiguous().t()  # columns contiguous
            y = torch.zeros((x.shape[1], nout), dtype=torch.float64, device=x.device).t()
        return self.matvec(x, y, trans=trans)

    def __matmul__(self, x):
        """A @ x as a new tensor: x a vector, or a matrix whose columns are
        right-hand sides (at most 64)."""
        return self._product(x, False)

    @property
    def T(self):
        """The transposed operator: op.T @ x computes A^T x."""
        return _Transposed(self)

    def tune(self, nrhs, stream=None):
        """Autotune the many-right-hand-side coupling product; returns its time in us."""
        best = _dbl()
        _check(h2b_op_tune(self.handle, int(nrhs), _stream_ptr(stream), ctypes.byref(best)))
        return best.value

    def set_geometry(self, verts, stream=None):
        """New vertex coordinates (same triangles); trees, boxes and
        interpolation points stay frozen."""
        v = np.ascontiguousarray(np.asarray(verts, dtype=np.float64).reshape(-1, 3))
        if len(v) != self.mesh.nv:
            raise ValueError("expected %d vertices" % self.mesh.nv)
        vx, vy, vz = (np.ascontiguousarray(v[:, d]) for d in range(3))
        _check(h2b_op_set_geometry(self.handle, _ptr(vx), _ptr(vy), _ptr(vz), _stream_ptr(stream)))

    def shape_grad(self, x, y, stream=None):
        """d(x^T G y)/d(vertex coordinates) as an (nv, 3) float64 CUDA tensor."""
        import torch
        g = torch.zeros((3, self.mesh.nv), dtype=torch.float64, device=x.device)
        _check(h2b_slp_shape_grad(self.handle, _vp(x.data_ptr()), _vp(y.data_ptr()), _vp(g[0].data_ptr()),
                                  _vp(g[1].data_ptr()), _vp(g[2].data_ptr()), _stream_ptr(stream)))
        return g.t()

    def set_timing(self, on=True):
        _check(h2b_op_set_timing(self.handle, int(bool(on))))

    def set_overlap(self, on=True):
        """Nearfield on its own stream beside the far field (default), or every
        phase on the caller's stream."""
        _check(h2b_op_set_overlap(self.handle, int(bool(on))))

    def phase_times(self):
        out = np.zeros(7)
        _check(h2b_op_phase_times(self.handle, _ptr(out)))
        return dict(zip(("gather", "forward", "coupling", "backward", "nearfield", "scatter", "total"), out))

    def mass_matvec(self, x, y, alpha=1.0, trans=False, stream=None):
        """y += alpha M x (x on the vertices, y on the triangles) or, with
        trans, y += alpha M^T x, for the mixed mass matrix of the mesh."""
        nin, nout = (self.mesh.nt, self.mesh.nv) if trans else (self.mesh.nv, self.mesh.nt)
        _vector(x, nin, "x")
        _vector(y, nout, "y")
        _check(h2b_mass_matvec(self.handle, int(bool(trans)), float(alpha), _vp(x.data_ptr()),
                               _vp(y.data_ptr()), _stream_ptr(stream)))
        return y

    def hypersingular_matvec(self, x, y, alpha=1.0, stream=None):
        """y += alpha W x for the hypersingular matrix W built from this
        single-layer operator (x, y: one entry per vertex)."""
        if self.kernel != H2B_SLP:
            raise ValueError("the hypersingular product needs the single-layer operator")
        _vector(x, self.mesh.nv, "x")
        _vector(y, self.mesh.nv, "y")
        _check(h2b_hypersingular_matvec(self.handle, float(alpha), _vp(x.data_ptr()), _vp(y.data_ptr()),
                                        _stream_ptr(stream)))
        return y

    def cg(self, b, x, tol=1e-8, max_iter=1000, check_every=8, use_graph=True, zero_guess=True,
           history=False, form="product", precond=None, hchol=None, stream=None):
        """Conjugate gradients for A x = b (A square, symmetric positive
        definite: the single-layer matrix G), or with form="hypersingular"
        for W x = b, W built from this single-layer operator; precond=
        "block_jacobi" preconditions with the inverse diagonal nearfield
        blocks of the leaves, precond="hchol" with the H-Cholesky factor
        `hchol` (an HChol of this operator).  x holds the
        initial guess (unless zero_guess) and receives the solution.  Returns
        a dict with iterations, status, rel_residual, solve_ms and, with
        history, the relative residual norms of iterations 0..iterations."""
        if form == "hypersingular":
            if self.kernel != H2B_SLP:
                raise ValueError("the hypersingular form needs the single-layer operator")
            n = self.mesh.nv
        else:
            if self.shape[0] != self.shape[1]:
                raise ValueError("conjugate gradients need a square operator")
            n = self.shape[0]
        _vector(b, n, "b")
        _vector(x, n, "x")
        p = h2b_cg_params()
        h2b_cg_params_default(ctypes.byref(p))
        p.tol, p.max_iter, p.check_every = float(tol), int(max_iter), int(check_every)
        p.use_graph, p.zero_guess = int(bool(use_graph)), int(bool(zero_guess))
        p.form = _FORMS[form]
        p.precond = _PRECONDS[precond]
        if precond == "hchol":
            if not isinstance(hchol, HChol):
                raise ValueError('precond="hchol" needs hchol=HChol(...)')
            p.hchol = hchol.handle
        r = h2b_cg_result()
        hist = np.zeros(max(int(max_iter), 0) + 1) if history else None
        _check(h2b_cg_solve(self.handle, _vp(b.data_ptr()), _vp(x.data_ptr()), ctypes.byref(p), ctypes.byref(r),
                            _ptr(hist) if history else None, _stream_ptr(stream)))
        out = dict(iterations=r.iterations, status=CG_STATUS.get(r.status, r.status),
                   rel_residual=r.rel_residual, solve_ms=r.solve_ms)
        if history:
            out["history"] = hist[:r.iterations + 1]
        return out

    def __del__(self, _destroy=h2b_op_destroy, _exiting=_EXITING):
        if getattr(self, "handle", None) and not _exiting[0]:
            _destroy(self.handle)
            self.handle = None


class _Transposed:
    """A^T of an Operator, for op.T @ x."""

    def __init__(self, op):
        self.op = op
        self.shape = (op.shape[1], op.shape[0])

    def __matmul__(self, x):
        return self.op._product(x, True)


class HChol:
    """H-Cholesky preconditioner G ~ L L^T of a single-layer operator,
    coarsened and factorised to the blockwise accuracy eps on the host; its
    substitutions z = (L L^T)^{-1} r run on the device (apply) or on the host
    (solve_host).  HChol(op, eps) builds it from an Operator;
    HChol.from_dense(blocks, A, eps) from a dense symmetric matrix on the
    blocks of one triangle tree (host only until the first apply)."""

    def __init__(self, op=None, eps=1e-3, stream=None, _handle=None, _keep=None):
        self.handle = None
        if _handle is not None:
            self.handle, self._keep = _handle, _keep
            return
        h = _vp()
        _check(h2b_hchol_build(op.handle, float(eps), ctypes.byref(h), _stream_ptr(stream)))
        self.handle, self._keep = h, op

    @classmethod
    def from_dense(cls, blocks, A, eps):
        A = np.ascontiguousarray(A, dtype=np.float64)
        h = _vp()
        _check(h2b_hchol_from_dense(blocks.handle, _ptr(A), float(eps), ctypes.byref(h)))
        return cls(_handle=h, _keep=blocks)

    def info(self):
        s = h2b_hchol_info()
        _check(h2b_hchol_get_info(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in s._fields_}

    def solve_host(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty_like(r)
        _check(h2b_hchol_solve_host(self.handle, _ptr(r), _ptr(z)))
        return z

    def apply(self, r, z, stream=None):
        n = self.info()["n"]
        _vector(r, n, "r")
        _vector(z, n, "z")
        _check(h2b_hchol_apply(self.handle, _vp(r.data_ptr()), _vp(z.data_ptr()), _stream_ptr(stream)))
        return z

    def __del__(self, _destroy=h2b_hchol_destroy, _exiting=_EXITING):
        if getattr(self, "handle", None) and not _exiting[0]:
            _destroy(self.handle)
            self.handle = None


def _vector(v, n, name):
    import torch
    if not isinstance(v, torch.Tensor) or v.dtype != torch.float64 or not v.is_cuda:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    if v.dim() != 1 or v.shape[0] != n or not v.is_contiguous():
        raise ValueError("%s must be a contiguous vector of length %d" % (name, n))


def dtn_rhs(K, u, stream=None):
    """Right-hand side (M/2 + K) u of the Dirichlet-to-Neumann system
    G t = (M/2 + K) u for the Dirichlet coefficients u (one per vertex) and
    the double-layer operator K: two library calls."""
    import torch
    b = torch.zeros(K.mesh.nt, dtype=torch.float64, device=u.device)
    K.mass_matvec(u, b, 0.5, stream=stream)
    K.matvec(u, b, stream=stream)
    return b


def ntd_rhs(K, t, stream=None):
    """Right-hand side (M^T/2 - K^T) t of the Neumann-to-Dirichlet system
    W u = (M^T/2 - K^T) t for the Neumann coefficients t (one per triangle)
    and the double-layer operator K: two library calls."""
    import torch
    b = torch.zeros(K.mesh.nv, dtype=torch.float64, device=t.device)
    K.mass_matvec(t, b, 0.5, trans=True, stream=stream)
    K.matvec(t, b, alpha=-1.0, trans=True, stream=stream)
    return b


class Batch:
    """Products of several operators captured into one HIP graph.

    ``Batch([(op, x, y), ...], alpha=1.0, trans=False)`` binds the device
    vectors; ``launch()`` replays y_i += alpha op_i x_i for all i."""

    def __init__(self, items, alpha=1.0, trans=False, stream=None):
        n = len(items)
        for op, x, y in items:
            nin = op.shape[0] if trans else op.shape[1]
            nout = op.shape[1] if trans else op.shape[0]
            if x.shape[0] != nin or y.shape[0] != nout:
                raise ValueError("vector length does not match its operator")
        self.items = list(items)  # keeps operators and vectors alive
        ops = (_vp * n)(*[op.handle for op, _, _ in items])
        tr = (ctypes.c_int * n)(*([int(bool(trans))] * n))
        al = (_dbl * n)(*([float(alpha)] * n))
        xs = (_vp * n)(*[x.data_ptr() for _, x, _ in items])
        ys = (_vp * n)(*[y.data_ptr() for _, _, y in items])
        ldx = (_i64 * n)(*[x.shape[0] if x.dim() == 1 else x.stride(1) for _, x, _ in items])
        ldy = (_i64 * n)(*[y.shape[0] if y.dim() == 1 else y.stride(1) for _, _, y in items])
        nr = (ctypes.c_int * n)(*[1 if x.dim() == 1 else x.shape[1] for _, x, _ in items])
        h = _vp()
        _check(h2b_batch_create(n, ops, tr, al, xs, ldx, ys, ldy, nr, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        _check(h2b_batch_launch(self.handle, _stream_ptr(stream)))

    def __del__(self, _destroy=h2b_batch_destroy, _exiting=_EXITING):
        if getattr(self, "handle", None) and not _exiting[0]:
            _destroy(self.handle)
            self.handle = None


class SlpBilinear(torch.autograd.Function):
    """b = x^T G(verts) y for the H^2 single-layer matrix of an Operator built
    with recompress_tol = 0; the cluster trees, boxes and interpolation points
    stay frozen at the operator's construction geometry.  The forward value
    comes from h2b_slp_bilinear (G y and the inner product in the library);
    the backward pass uses the library's adjoint kernels for d b / d verts and
    G y, G^T x for the vectors, scaled by the incoming gradient (autograd's
    chain rule).

        b = SlpBilinear.apply(verts, x, y, op)"""

    @staticmethod
    def forward(ctx, verts, x, y, op):
        op.set_geometry(verts.detach().cpu().numpy())
        gy = torch.empty_like(x)
        b = torch.empty((), dtype=torch.float64, device=x.device)
        _vector(x, op.mesh.nt, "x")
        _vector(y, op.mesh.nt, "y")
        _check(h2b_slp_bilinear(op.handle, _vp(x.data_ptr()), _vp(y.data_ptr()), _vp(gy.data_ptr()),
                                _vp(b.data_ptr()), _stream_ptr(None)))
        ctx.save_for_backward(x, y, gy)
        ctx.op = op
        ctx.vspec = (verts.device, verts.dtype)
        return b

    @staticmethod
    def backward(ctx, gout):
        x, y, gy = ctx.saved_tensors
        op = ctx.op
        gverts = op.shape_grad(x, y)
        gtx = torch.zeros_like(y)
        op.matvec(x, gtx, trans=True)
        gv = (gout * gverts).to(device=ctx.vspec[0], dtype=ctx.vspec[1])
        return gv, gout * gy, gout * gtx, None
