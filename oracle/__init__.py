"""Test infrastructure only: the CPU double-precision oracle.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
and does not import it.

* ``bem_oracle.c`` -- dense Galerkin entries of the single-layer matrix G and
  the double-layer matrix K (Section 1, eqs. (slp), (dlp)) by singular
  (Sauter-Schwab) and regular Gauss quadrature of triangle pairs.
* ``h2.py`` -- cluster tree, block tree and the interpolation-based H^2
  approximation (Sections 2 and 3) written out as dense matrices, for small
  meshes.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bem_oracle.c")
_LIB = os.path.join(_HERE, "libbem_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE double)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        L.orc_gauss_legendre01.argtypes = [i32, vp, vp]
        L.orc_slp_dense.argtypes = [i64, vp, i64, vp, i32, vp]
        L.orc_dlp_dense.argtypes = [i64, vp, i64, vp, i32, vp]
        L.orc_slp_rows.argtypes = [i64, vp, i64, vp, i32, i32, i64, vp, vp, vp]
        L.orc_dlp_rows.argtypes = [i64, vp, i64, vp, i32, i32, i64, vp, vp, vp]
        L.orc_slp_block.argtypes = [i64, vp, i64, vp, i32, i64, vp, i64, vp, vp]
        L.orc_dlp_block.argtypes = [i64, vp, i64, vp, i32, i64, vp, i64, vp, vp]
        L.orc_slp_entry.argtypes = [i64, vp, i64, vp, i32, i64, i64]
        L.orc_slp_entry.restype = dbl
        L.orc_dlp_pair.argtypes = [i64, vp, i64, vp, i32, i64, i64, vp]
        L.orc_set_threads.argtypes = [i32]
        L.orc_get_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _mesh(verts, tris):
    V = np.ascontiguousarray(verts, dtype=np.float64).reshape(-1, 3)
    T = np.ascontiguousarray(tris, dtype=np.int32).reshape(-1, 3)
    return V, T


def set_threads(n):
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def gauss_legendre01(q):
    t = np.zeros(q)
    w = np.zeros(q)
    if lib().orc_gauss_legendre01(q, _ptr(t), _ptr(w)) != 0:
        raise ValueError("q out of range")
    return t, w


def slp_dense(verts, tris, q):
    V, T = _mesh(verts, tris)
    G = np.zeros((len(T), len(T)))
    if lib().orc_slp_dense(len(V), _ptr(V), len(T), _ptr(T), q, _ptr(G)) != 0:
        raise ValueError("bad quadrature order")
    return G


def dlp_dense(verts, tris, q):
    V, T = _mesh(verts, tris)
    K = np.zeros((len(T), len(V)))
    if lib().orc_dlp_dense(len(V), _ptr(V), len(T), _ptr(T), q, _ptr(K)) != 0:
        raise ValueError("bad quadrature order")
    return K


def slp_rows(verts, tris, q, rows, x, trans=False):
    V, T = _mesh(verts, tris)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == (len(T),)
    y = np.zeros(len(rows))
    if lib().orc_slp_rows(len(V), _ptr(V), len(T), _ptr(T), q, int(bool(trans)),
                          len(rows), _ptr(rows), _ptr(x), _ptr(y)) != 0:
        raise ValueError("bad quadrature order")
    return y


def dlp_rows(verts, tris, q, rows, x, trans=False):
    V, T = _mesh(verts, tris)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    assert x.shape == ((len(T),) if trans else (len(V),))
    y = np.zeros(len(rows))
    if lib().orc_dlp_rows(len(V), _ptr(V), len(T), _ptr(T), q, int(bool(trans)),
                          len(rows), _ptr(rows), _ptr(x), _ptr(y)) != 0:
        raise ValueError("bad quadrature order")
    return y


def slp_block(verts, tris, q, rows, cols):
    """Dense G entries G[rows][:, cols] (rows and columns are triangles)."""
    V, T = _mesh(verts, tris)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros((len(rows), len(cols)))
    if lib().orc_slp_block(len(V), _ptr(V), len(T), _ptr(T), q, len(rows), _ptr(rows), len(cols),
                           _ptr(cols), _ptr(out)) != 0:
        raise ValueError("bad quadrature order or index")
    return out


def dlp_block(verts, tris, q, rows, cols):
    """Dense K entries K[rows][:, cols] (rows triangles, columns vertices)."""
    V, T = _mesh(verts, tris)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros((len(rows), len(cols)))
    if lib().orc_dlp_block(len(V), _ptr(V), len(T), _ptr(T), q, len(rows), _ptr(rows), len(cols),
                           _ptr(cols), _ptr(out)) != 0:
        raise ValueError("bad quadrature order or index")
    return out


def slp_entry(verts, tris, q, i, j):
    V, T = _mesh(verts, tris)
    return float(lib().orc_slp_entry(len(V), _ptr(V), len(T), _ptr(T), q, i, j))


def dlp_pair(verts, tris, q, i, j):
    """Contributions of triangle pair (i, j) to K: entry c goes to column tris[j][c]."""
    V, T = _mesh(verts, tris)
    val = np.zeros(3)
    if lib().orc_dlp_pair(len(V), _ptr(V), len(T), _ptr(T), q, i, j, _ptr(val)) != 0:
        raise ValueError("bad arguments")
    return val
